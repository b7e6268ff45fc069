"""Seeded synthetic TT inputs shared by the oracle tests and the HIP path.

This module only draws random numbers and lays them out; it holds none of the
TT arithmetic (no sums, products, orthonormalization or rounding).  Each side
builds its own working tensors (e.g. ``X = A + B``) with its own ``add``.

Recipe (the paper's experiments use random TT tensors, §4.2):
* every core is i.i.d. standard normal float64, drawn from
  ``numpy.random.default_rng(SeedSequence([201106532, cfg, tt, role, n]))``
  (role Y=0, A=1, B=2, C=3, E=4), filled in the paper's core layout
  (entry (a, i, b) at a + R_{n-1}(i + I_n b), i.e. Fortran order);
* ``scaled`` multiplies core n by 1/sqrt(R_{n-1} I_n) so that E||X||^2 = 1;
* ``first_core_factor`` multiplies core 1 (used for the 1e-6 / 1e-9 parts);
* ``rank_weights`` multiplies entry (a, i, b) by 2^-b on cores 1..N-1
  (decaying slice weights over the trailing rank index).

Cores are returned as Fortran-ordered numpy arrays of shape (R_{n-1}, I_n, R_n).
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Sequence

import numpy as np

SEED_ROOT = 201106532
ROLE = {"Y": 0, "A": 1, "B": 2, "C": 3, "E": 4}


def core_rng(cfg: int, tt: int, role: str, n: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, cfg, tt, ROLE[role], n]))


def _one_core(cfg, tt, role, n, r0, I, r1, scaled, factor, weights):
    rng = core_rng(cfg, tt, role, n)
    flat = np.empty(r0 * I * r1, dtype=np.float64)
    rng.standard_normal(out=flat)
    core = flat.reshape(r0, I, r1, order="F")
    s = factor
    if scaled:
        s /= math.sqrt(r0 * I)
    if s != 1.0:
        core *= s
    if weights:
        core *= (2.0 ** -np.arange(r1, dtype=np.float64))[None, None, :]
    return core


def random_tt(cfg: int, tt: int, role: str, I: Sequence[int], r: Sequence[int],
              scaled: bool = False, first_core_factor: float = 1.0,
              rank_weights: bool = False, threads: Optional[int] = None) -> List[np.ndarray]:
    """Random TT with mode sizes ``I`` and interior ranks ``r`` (len(I)-1 values)."""
    N = len(I)
    R = [1] + list(r) + [1]
    assert len(R) == N + 1
    jobs = []
    for n in range(N):
        factor = first_core_factor if n == 0 else 1.0
        w = rank_weights and n < N - 1
        jobs.append((cfg, tt, role, n, R[n], int(I[n]), R[n + 1], scaled, factor, w))
    total = sum(j[4] * j[5] * j[6] for j in jobs)
    if threads is None:
        threads = min(16, os.cpu_count() or 1) if total > 4_000_000 else 1
    if threads <= 1:
        return [_one_core(*j) for j in jobs]
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda j: _one_core(*j), jobs))


# ---------------------------------------------------------------------------
# The five workloads.  ``I_override`` shrinks the mode size (bounded samples,
# parity sizes); everything else keeps the workload's structure.
# ---------------------------------------------------------------------------

WORKLOADS = {
    0: "Y+Y: N=4, I=64, Y ranks 5 (unscaled N(0,1)), tol 1e-10, RLR",
    1: "A+B: N=16, I=262144, A,B ranks 20 (scaled), formal ranks 40, tol 1e-8",
    2: "A+B+1e-6*C: N=16, I=262144, A,B ranks 20, C rank 10, formal ranks 50, tol 1e-8",
    3: "512 x (Y+Y+E): N=8, I log-uniform [64,4096], Y ranks in 1..31, E rank 2 scaled 1e-9, tol 1e-7",
    4: "A*B (Hadamard): N=10, I=16384, A,B ranks 16 with 2^-b rank weights, formal ranks 256, tol 1e-6",
}

TOL = {0: 1e-10, 1: 1e-8, 2: 1e-8, 3: 1e-7, 4: 1e-6}


def yy_small(I_override: Optional[int] = None) -> Dict:
    I = I_override or 64
    Y = random_tt(0, 0, "Y", [I] * 4, [5, 5, 5], scaled=False)
    return {"Y": Y, "tol": TOL[0]}


def sum_r40(I_override: Optional[int] = None, N: int = 16, r: int = 20) -> Dict:
    I = I_override or 262144
    A = random_tt(1, 0, "A", [I] * N, [r] * (N - 1), scaled=True)
    B = random_tt(1, 0, "B", [I] * N, [r] * (N - 1), scaled=True)
    return {"A": A, "B": B, "tol": TOL[1]}


def sum_r50(I_override: Optional[int] = None, N: int = 16) -> Dict:
    I = I_override or 262144
    A = random_tt(2, 0, "A", [I] * N, [20] * (N - 1), scaled=True)
    B = random_tt(2, 0, "B", [I] * N, [20] * (N - 1), scaled=True)
    C = random_tt(2, 0, "C", [I] * N, [10] * (N - 1), scaled=True, first_core_factor=1e-6)
    return {"A": A, "B": B, "C": C, "tol": TOL[2]}


def batched_shapes(count: int = 512, N: int = 8):
    """Per-TT mode sizes round(exp(U[ln 64, ln 4096])) and Y ranks uniform in {1..31}."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 3, 10**6]))
    shapes = []
    for _ in range(count):
        I = [int(round(math.exp(rng.uniform(math.log(64), math.log(4096))))) for _ in range(N)]
        r = [int(x) for x in rng.integers(1, 32, size=N - 1)]
        shapes.append((I, r))
    return shapes


def batched(count: int = 512, N: int = 8, I_cap: Optional[int] = None) -> Dict:
    shapes = batched_shapes(count, N)
    Ys, Es = [], []
    for t, (I, r) in enumerate(shapes):
        if I_cap:
            I = [min(x, I_cap) for x in I]
        Ys.append(random_tt(3, t, "Y", I, r, scaled=True))
        Es.append(random_tt(3, t, "E", I, [2] * (N - 1), scaled=True, first_core_factor=1e-9))
    return {"Y": Ys, "E": Es, "tol": TOL[3]}


def hadamard_r256(I_override: Optional[int] = None, N: int = 10, r: int = 16) -> Dict:
    I = I_override or 16384
    A = random_tt(4, 0, "A", [I] * N, [r] * (N - 1), scaled=True, rank_weights=True)
    B = random_tt(4, 0, "B", [I] * N, [r] * (N - 1), scaled=True, rank_weights=True)
    return {"A": A, "B": B, "tol": TOL[4]}


def core_bytes_of_sum(I: Sequence[int], r: Sequence[int]) -> int:
    """Bytes of a TT with the given modes and interior ranks (layout arithmetic only)."""
    R = [1] + list(r) + [1]
    return int(sum(8 * R[n] * I[n] * R[n + 1] for n in range(len(I))))
