"""GPU parity of the basic TT operations against the FP64 oracle, through the
C ABI (libttr.so via its ctypes binding)."""
import math

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def rand_tt(rng, I, r, scale=1.0):
    R = [1] + list(r) + [1]
    return [np.asfortranarray(scale * rng.standard_normal((R[n], I[n], R[n + 1]))) for n in range(len(I))]


SHAPES = [
    ([5, 4, 6], [3, 2]),
    ([3, 7, 2, 4], [2, 5, 3]),
    ([6], []),
    ([4, 1, 5], [2, 2]),                   # I_n = 1
    ([300, 257, 129], [7, 9]),             # several chunks and a ragged tail
    ([2000, 3, 1500], [17, 23]),
]


@pytest.fixture(scope="module")
def h(ttr):
    hd = ttr.Handle(0)
    yield hd
    hd.close()


@pytest.mark.parametrize("I,r", SHAPES)
def test_add_bitwise(ttr, h, I, r):
    print(f"add I={I} r={r}", flush=True)
    rng = np.random.default_rng(100)
    X = rand_tt(rng, I, r)
    Y = rand_tt(rng, I, [x + 1 for x in r])
    Z = h.add(1.25, ttr.TT.from_numpy(X), -0.5, ttr.TT.from_numpy(Y)).to_numpy()
    ref = O.add(1.25, X, -0.5, Y)
    assert O.ranks(Z) == O.ranks(ref)
    for z, zr in zip(Z, ref):
        assert np.array_equal(z, zr)


@pytest.mark.parametrize("I,rx,ry", [([64, 50, 32, 80], [4, 6, 2], [2, 4, 8]),
                                     ([33, 50, 32, 81], [4, 6, 2], [2, 4, 8]),
                                     ([40, 40], [20], [20])])
def test_add_bitwise_even_ranks(ttr, h, I, rx, ry):
    # even ranks (and even I on the first core) take the paired 16-byte kernel
    print(f"add even ranks I={I} rx={rx} ry={ry}", flush=True)
    rng = np.random.default_rng(108)
    X = rand_tt(rng, I, rx)
    Y = rand_tt(rng, I, ry)
    Z = h.add(0.75, ttr.TT.from_numpy(X), -1.5, ttr.TT.from_numpy(Y)).to_numpy()
    ref = O.add(0.75, X, -1.5, Y)
    assert O.ranks(Z) == O.ranks(ref)
    for z, zr in zip(Z, ref):
        assert np.array_equal(z, zr)


@pytest.mark.parametrize("I,r", SHAPES)
def test_hadamard_bitwise(ttr, h, I, r):
    print(f"hadamard I={I} r={r}", flush=True)
    rng = np.random.default_rng(101)
    X = rand_tt(rng, I, r)
    Y = rand_tt(rng, I, [max(1, x - 1) for x in r])
    Z = h.hadamard(ttr.TT.from_numpy(X), ttr.TT.from_numpy(Y)).to_numpy()
    ref = O.hadamard(X, Y)
    assert O.ranks(Z) == O.ranks(ref)
    for z, zr in zip(Z, ref):
        assert np.array_equal(z, zr)


@pytest.mark.parametrize("I,r", SHAPES)
def test_dot_and_norms(ttr, h, I, r):
    print(f"dot/norm I={I} r={r}", flush=True)
    rng = np.random.default_rng(102)
    X = rand_tt(rng, I, r)
    Y = rand_tt(rng, I, [x + 2 for x in r])
    gx, gy = ttr.TT.from_numpy(X), ttr.TT.from_numpy(Y)
    ref = O.dot(X, Y)
    scale = O.norm_ortho(X) * O.norm_ortho(Y)
    assert abs(h.dot(gx, gy) - ref) <= 1e-12 * scale
    n = O.norm_ortho(X)
    assert abs(h.norm(gx, "gram") - n) <= 1e-12 * n
    assert abs(h.norm(gx, "sym") - n) <= 1e-12 * n
    assert abs(h.norm(gx, "ortho") - n) <= 1e-12 * n


DOT_SHAPES = [
    ([3000, 2000, 2500], [40, 33], [64, 9]),         # different tile counts on the two sides
    ([700, 1, 800, 2], [40, 64, 5], [3, 17, 48]),
    ([5000, 4000], [64], [64]),
    ([257, 129, 65, 33], [1, 16, 17], [31, 2, 1]),
]


@pytest.mark.parametrize("I,rx,ry", DOT_SHAPES)
def test_dot_matrix_cores(ttr, h, I, rx, ry):
    # the inner-product steps on the matrix cores: all rank combinations up
    # to 64, ragged slices, both argument orders
    print(f"dot I={I} rx={rx} ry={ry}", flush=True)
    rng = np.random.default_rng(106)
    X = rand_tt(rng, I, rx, scale=0.2)
    Y = rand_tt(rng, I, ry, scale=0.2)
    gx, gy = ttr.TT.from_numpy(X), ttr.TT.from_numpy(Y)
    ref = O.dot(X, Y)
    scale = O.norm_ortho(X) * O.norm_ortho(Y)
    assert abs(h.dot(gx, gy) - ref) <= 1e-12 * scale
    assert abs(h.dot(gy, gx) - ref) <= 1e-12 * scale
    n = O.norm_ortho(X)
    assert abs(h.norm(gx, "gram") - n) <= 1e-12 * n


SYM_SHAPES = [
    ([4000, 3000, 2500, 2000], [16, 33, 64]),      # every tile count, ragged tails
    ([700, 1, 800, 2, 600], [40, 64, 48, 12]),     # R_n > R_{n-1} I_n: singular W_2, W_3
    ([1000, 1200], [1]),
    ([513, 64, 257], [64, 64]),
]


@pytest.mark.parametrize("I,r", SYM_SHAPES)
def test_norm_sym_matches_oracle(ttr, h, I, r):
    # symmetric inner-product norm: pivoted Cholesky factors made triangular,
    # the half-skipping matrix-core Gram; parity with the oracle's form and
    # with the other two methods
    print(f"norm sym I={I} r={r}", flush=True)
    rng = np.random.default_rng(104)
    X = rand_tt(rng, I, r, scale=0.1)
    gx = ttr.TT.from_numpy(X)
    ref = O.norm_gram_sym(X)
    got = h.norm(gx, "sym")
    assert abs(got - ref) <= 1e-12 * ref
    assert abs(h.norm(gx, "gram") - ref) <= 1e-12 * ref
    assert abs(h.norm(gx, "ortho") - ref) <= 1e-12 * ref


def test_norm_sym_rank_deficient_and_nonfinite(ttr, h):
    print("norm sym of Y + Y, zero and non-finite tensors", flush=True)
    rng = np.random.default_rng(105)
    Y = rand_tt(rng, [300, 200, 250, 100], [9, 20, 11])
    X = O.add(1.0, Y, 1.0, Y)                       # every W_n has half rank
    n = np.sqrt(O.dot(Y, Y))
    assert abs(h.norm(ttr.TT.from_numpy(X), "sym") - 2 * n) <= 1e-12 * n
    Z = [np.zeros_like(c) for c in Y]
    assert h.norm(ttr.TT.from_numpy(Z), "sym") == 0.0
    Y[2][4, 17, 3] = np.inf
    assert math.isnan(h.norm(ttr.TT.from_numpy(Y), "sym"))
    assert not math.isfinite(h.norm(ttr.TT.from_numpy(Y), "gram"))


def test_norm_ortho_small_difference(ttr, h):
    # ||X - (X + 1e-9 Z)|| = 1e-9 ||Z||: the orthonormal route resolves it,
    # where sqrt(<D, D>) of the difference TT loses it to cancellation (§3.2.4).
    print("norm of a difference tensor", flush=True)
    rng = np.random.default_rng(103)
    I = [50, 60, 40, 30]
    X = rand_tt(rng, I, [4, 5, 3])
    Z = rand_tt(rng, I, [2, 2, 2])
    Xp = O.add(1.0, X, 1e-9, Z)
    D = O.add(1.0, Xp, -1.0, X)
    ref = 1e-9 * O.norm_ortho(Z)
    got = h.norm(ttr.TT.from_numpy(D), "ortho")
    assert abs(got - ref) <= 1e-6 * ref


@pytest.mark.parametrize("side", ["right", "left"])
@pytest.mark.parametrize("I,r", SHAPES)
def test_orthogonalize(ttr, h, side, I, r):
    print(f"orthogonalize {side} I={I} r={r}", flush=True)
    rng = np.random.default_rng(104)
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
    # generic inputs keep their ranks unless a thin unfolding caps them
    assert O.ranks(Y) == O.ranks(O.orthogonalize(X, side))


def test_orthogonalize_rank_deficient(ttr, h):
    # Y + Y: every unfolding is exactly rank deficient; the rank-revealing
    # factorization keeps the numerical rank and preserves the tensor.
    print("orthogonalize Y+Y", flush=True)
    rng = np.random.default_rng(105)
    Yc = rand_tt(rng, [40, 30, 50, 20], [4, 6, 3])
    X = O.add(1.0, Yc, 1.0, Yc)
    g = ttr.TT.from_numpy(X)
    h.orthogonalize(g, "right")
    Y = g.to_numpy()
    assert O.ranks(Y) == [1, 4, 6, 3, 1]
    assert O.diff_norm(Y, X) <= 1e-13 * O.norm_ortho(X) * 4
    # against the oracle's orthonormalization (Householder, formal ranks 8, 12,
    # 6 with rounding-level directions): the same tensor, and the GPU's ranks
    # are the numerical ranks of the tensor's unfoldings (the TT ranks, §2.1)
    ref = O.orthogonalize(X, "right")
    assert O.ranks(ref) == [1, 8, 12, 6, 1]
    assert O.diff_norm(Y, ref) <= 1e-12 * O.norm_ortho(ref)
    full = O.full(X)
    num = [1]
    for n in range(1, 4):
        s = np.linalg.svd(full.reshape(int(np.prod(full.shape[:n])), -1), compute_uv=False)
        num.append(int(np.sum(s > 1e-12 * s[0])))
    assert O.ranks(Y) == num + [1]
    for n in range(1, 4):
        Hn = O.H(Y[n])
        assert np.linalg.norm(Hn @ Hn.T - np.eye(Hn.shape[0])) < 1e-12


def _offset_tt(ttr, cores_np=None, I=None, caps=None):
    """A TT whose device cores start 8 bytes into their allocations (8-byte
    aligned, not 16): from host cores, or empty with the given capacities."""
    import torch
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


@pytest.mark.parametrize("rank", [6, 80])
def test_cores_not_16_byte_aligned(ttr, h, rank):
    # inputs and outputs 8 bytes into their allocations: the 16-byte access
    # paths (paired sums, paired Gram loads, streaming copies) must take their
    # scalar forms; every result against the oracle
    print(f"cores at 8-byte offsets, sum ranks {rank}", flush=True)
    rng = np.random.default_rng(108)
    I = [40, 30, 50, 20]
    N = len(I)
    A = rand_tt(rng, I, [rank // 2] * (N - 1))
    B = rand_tt(rng, I, [rank // 2] * (N - 1))
    gA, gB = _offset_tt(ttr, A), _offset_tt(ttr, B)
    assert all(c.data_ptr() % 16 == 8 for c in gA.cores)
    Rs = [1] + [rank] * (N - 1) + [1]
    caps = [Rs[n] * I[n] * Rs[n + 1] for n in range(N)]
    out = _offset_tt(ttr, I=I, caps=caps)
    Z = h.add(1.0, gA, -0.5, gB, out=out)
    X = O.add(1.0, A, -0.5, B)
    for g, e in zip(Z.to_numpy(), X):
        assert np.array_equal(g, e)
    if rank <= 16:
        Hc = [R0 * R1 for R0, R1 in zip([1] + [rank // 2] * (N - 1) + [1], [1] + [rank // 2] * (N - 1) + [1])]
        hcaps = [Hc[n] * I[n] * Hc[n + 1] for n in range(N)]
        Hg = h.hadamard(gA, gB, out=_offset_tt(ttr, I=I, caps=hcaps))
        for g, e in zip(Hg.to_numpy(), O.hadamard(A, B)):
            assert np.array_equal(g, e)
    nrm2 = O.dot(X, X)
    assert math.isclose(h.dot(Z, Z), nrm2, rel_tol=1e-12)
    for direction in ("RLR", "LRL", "RLR_EXPLICIT"):
        Y = h.round(Z, 1e-8, direction, out=_offset_tt(ttr, I=I, caps=caps))
        ref = O.round_tt(X, 1e-8, "LRL" if direction == "LRL" else "RLR")
        got = Y.to_numpy()
        assert O.ranks(got) == O.ranks(ref), direction
        assert O.diff_norm(got, ref) <= 1e-10 * O.norm_ortho(ref), direction
    T = h.orthogonalize(_offset_tt(ttr, X), "right")
    assert O.diff_norm(T.to_numpy(), X) <= 1e-12 * math.sqrt(nrm2) * N


def test_argument_errors(ttr, h):
    rng = np.random.default_rng(106)
    X = ttr.TT.from_numpy(rand_tt(rng, [5, 6], [3]))
    Y = ttr.TT.from_numpy(rand_tt(rng, [5, 7], [3]))
    with pytest.raises(ttr.TTRError) as e:
        h.add(1.0, X, 1.0, Y)
    assert e.value.code == 2  # shape
    with pytest.raises(ttr.TTRError) as e:
        h.round(X, -1.0)
    assert e.value.code == 1
    with pytest.raises(ttr.TTRError) as e:
        h.round(X, float("nan"))
    assert e.value.code == 1
    small = ttr.TT.empty([5, 6], [1, 1], X.cores[0].device)
    with pytest.raises(ttr.TTRError) as e:
        h.round(X, 1e-3, out=small)
    assert e.value.code == 3  # capacity
    # ranks above TTR_MAX_RANK_LARGE: every entry point that takes ranks
    big = ttr.TT.from_numpy(rand_tt(rng, [3, 3], [257]))
    with pytest.raises(ttr.TTRError) as e:
        h.round(big, 1e-3)
    assert e.value.code == 7
    with pytest.raises(ttr.TTRError) as e:
        h.orthogonalize(big, "right")
    assert e.value.code == 7
    with pytest.raises(ttr.TTRError) as e:
        h.dot(big, big)
    assert e.value.code == 7
    with pytest.raises(ttr.TTRError) as e:
        h.norm(big, "ortho")
    assert e.value.code == 7


def test_nonfinite_input_reports_numerical(ttr, h):
    rng = np.random.default_rng(107)
    X = rand_tt(rng, [20, 30, 20], [3, 4])
    X[1][0, 3, 1] = np.nan
    with pytest.raises(ttr.TTRError) as e:
        h.round(ttr.TT.from_numpy(X), 1e-6)
    assert e.value.code == 6


def test_workspace_through_caller_allocator(ttr):
    # ttr_set_allocator: every workspace comes from (and goes back to) the
    # caller's allocator -- here torch's caching allocator -- and results are
    # those of the default allocator
    import torch
    print("allocator hook", flush=True)
    rng = np.random.default_rng(110)
    I, r = [300, 257, 129, 64], [9, 12, 7]
    X = rand_tt(rng, I, r)
    tol = 1e-3
    ref_h = ttr.Handle(0)
    ref = ref_h.round(ttr.TT.from_numpy(X), tol, "RLR").to_numpy()
    ref_h.close()
    calls = {"alloc": 0, "free": 0}
    h = ttr.Handle(0)
    stream = torch.cuda.current_stream(0)

    def alloc(n):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(n, 0, stream)

    def free(p):
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    h.set_allocator(alloc, free)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    got = h.round(ttr.TT.from_numpy(X), tol, "RLR").to_numpy()
    torch.cuda.synchronize()
    assert calls["alloc"] >= 1
    assert torch.cuda.memory_allocated(0) > before  # the workspace is torch memory
    assert O.ranks(got) == O.ranks(ref)
    assert O.diff_norm(got, ref) <= 1e-12 * O.norm_ortho(ref)
    # back to hipMalloc: the workspace is returned to torch first
    h.set_allocator(None, None)
    assert calls["free"] == calls["alloc"]
    again = h.round(ttr.TT.from_numpy(X), tol, "RLR").to_numpy()
    assert O.diff_norm(again, ref) <= 1e-12 * O.norm_ortho(ref)
    with pytest.raises(ValueError):
        h.set_allocator(alloc, None)
    h.close()


def test_allocator_failure_reports_alloc(ttr):
    # an allocator that returns NULL makes the call that needs memory fail
    # with TTR_ERR_ALLOC; a later default allocator works again
    print("allocator failure", flush=True)
    rng = np.random.default_rng(111)
    X = rand_tt(rng, [50, 40, 30], [6, 5])
    h = ttr.Handle(0)
    h.set_allocator(lambda n: 0, lambda p: None)
    with pytest.raises(ttr.TTRError) as e:
        h.round(ttr.TT.from_numpy(X), 1e-6, "RLR")
    assert e.value.code == 4
    h.set_allocator(None, None)
    Y = h.round(ttr.TT.from_numpy(X), 1e-6, "RLR").to_numpy()
    assert O.ranks(Y) == [1, 6, 5, 1]
    h.close()


def _band(rng, n, kl, ku):
    """A random n x n matrix with kl sub- and ku super-diagonals, dense and in
    band storage (torch shape (n, kl + ku + 1): row j holds column j)."""
    A = rng.standard_normal((n, n))
    i, j = np.indices((n, n))
    A[(i - j > kl) | (j - i > ku)] = 0.0
    ld = kl + ku + 1
    AB = np.zeros((n, ld))
    for jj in range(n):
        for ii in range(max(0, jj - ku), min(n, jj + kl + 1)):
            AB[jj, ku + ii - jj] = A[ii, jj]
    return A, AB


KRON_CASES = [
    ([300, 257, 129, 64], [9, 33, 7], [(1, 1), (0, 2), (3, 0), (1, 1)]),
    ([40, 35, 50], [64, 64], [(39, 39), (2, 5), (49, 49)]),          # dense A_1 and A_3
    ([1000, 20, 800], [5, 256], [(1, 1), (19, 0), (2, 2)]),           # a rank-256 core
    ([7, 1, 9], [3, 3], [(6, 6), (0, 0), (1, 3)]),                    # I_n = 1
]


@pytest.mark.parametrize("I,r,bands", KRON_CASES)
def test_apply_kron_matches_oracle(ttr, h, I, r, bands):
    import torch
    print(f"Kronecker operator I={I} r={r} bands={bands}", flush=True)
    rng = np.random.default_rng(120)
    X = rand_tt(rng, I, r)
    dense, band = zip(*[_band(rng, n, kl, ku) for n, (kl, ku) in zip(I, bands)])
    AB = [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in band]
    Y = h.apply_kron(AB, [b[0] for b in bands], [b[1] for b in bands], ttr.TT.from_numpy(X)).to_numpy()
    ref = O.apply_kron(list(dense), X)
    assert O.ranks(Y) == O.ranks(X)
    for n, (y, yr) in enumerate(zip(Y, ref)):
        assert np.max(np.abs(y - yr)) <= 1e-13 * max(np.max(np.abs(yr)), 1e-300), n


def test_apply_kron_sum_and_round(ttr, h):
    # the Krylov building block: Y = (A_1 (x) ... (x) A_N) X + X, then rounding,
    # against the oracle's same three steps
    print("Kronecker operator, sum and rounding", flush=True)
    rng = np.random.default_rng(121)
    I = [200, 150, 180, 120]
    X = rand_tt(rng, I, [6, 8, 5])
    lap = []
    for n in I:   # 1-D Laplacian stencil (tridiagonal)
        A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        lap.append(A)
    band = [np.stack([-np.ones(n), 2.0 * np.ones(n), -np.ones(n)], axis=1) for n in I]  # (ku=1: row j = [A(j-1,j), A(j,j), A(j+1,j)])
    AB = [torch_tensor(b) for b in band]
    gX = ttr.TT.from_numpy(X)
    gY = h.apply_kron(AB, [1] * len(I), [1] * len(I), gX)
    gS = h.add(1.0, gY, 1.0, gX)
    got = h.round(gS, 1e-10).to_numpy()
    S = O.add(1.0, O.apply_kron(lap, X), 1.0, X)
    ref = O.round_tt(S, 1e-10)
    assert O.ranks(got) == O.ranks(ref)
    assert O.diff_norm(got, ref) <= 1e-10 * O.norm_ortho(ref)


def torch_tensor(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()
