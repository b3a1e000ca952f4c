"""Shared test helpers: unit roundoffs, tolerances, host/device plane transfers."""
from __future__ import annotations

import numpy as np

# unit roundoff per format as used by the acceptance bounds (106/159/212-bit formats
# with slack for the per-operation error bounds)
U_FMT = {2: 2.0 ** -104, 3: 2.0 ** -157, 4: 2.0 ** -209}


def to_dev(P: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(P)).to("cuda")


def to_host(T) -> np.ndarray:
    return T.detach().cpu().numpy().copy()


def cabs1_hi(P: np.ndarray) -> np.ndarray:
    """|Re| + |Im| of the leading components, as a (rows, cols) real matrix."""
    return (np.abs(P[0, 0]) + np.abs(P[1, 0])).T


def gemm_tol(A, B, Cm, opA, opB, C, k):
    """Elementwise bound 4 (k + 4) u (sum_t cabs1(a) cabs1(b) + cabs1(c))."""
    a = cabs1_hi(A)
    b = cabs1_hi(B)
    if opA != "N":
        a = a.T
    if opB != "N":
        b = b.T
    S = a @ b
    if Cm is not None:
        S = S + cabs1_hi(Cm)
    return 4 * (k + 4) * U_FMT[C] * S


def exact_lu_case(n, C, seed, ld=None):
    """A = P^T L U whose elimination is exact in binary64 (see test_oracle_lu)."""
    import synthgen

    rng = np.random.default_rng(seed)
    L = np.eye(n, dtype=complex)
    U = np.zeros((n, n), dtype=complex)
    for i in range(n):
        for j in range(n):
            if i > j:
                L[i, j] = (rng.integers(-64, 65) + 1j * rng.integers(-64, 65)) / 256.0
            elif i < j:
                U[i, j] = (rng.integers(-256, 257) + 1j * rng.integers(-256, 257)) / 256.0
        e = 2.0 ** int(rng.integers(-2, 3))
        kind = rng.integers(0, 3)
        sr, si = rng.choice([-1, 1]), rng.choice([-1, 1])
        U[i, i] = e * (sr if kind == 0 else (1j * si if kind == 1 else sr + 1j * si))
    perm = rng.permutation(n)
    LU = L @ U
    A = np.zeros_like(LU)
    A[perm] = LU
    pos = list(perm)
    at = {pos[i]: i for i in range(n)}
    ipiv = []
    for k in range(n):
        p = pos[k]
        ipiv.append(p + 1)
        other = at[k]
        at[k], at[p] = k, other
        pos[k], pos[other] = k, p
    return synthgen.planes_from_complex(A, C, ld), L, U, np.array(ipiv, dtype=np.int32)


def pivot_gaps_clear(LUh: np.ndarray, rel=1e-12) -> int:
    """Number of leading columns whose pivot beat every other candidate by a relative
    cabs1 margin > rel, judged from the leading components of the factors."""
    n = min(LUh.shape)
    for k in range(n - 1):
        ukk = LUh[k, k]
        cp = abs(ukk.real) + abs(ukk.imag)
        col = LUh[k + 1:, k] * ukk
        if col.size and (np.abs(col.real) + np.abs(col.imag)).max() > cp * (1 - rel):
            return k
    return n
