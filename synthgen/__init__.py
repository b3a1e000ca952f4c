"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU oracle.

This module only draws random numbers and lays them out; it holds none of the LU
method's arithmetic.  All matrices are complex multi-component planes in the library's
layout: float64 numpy arrays of shape ``(2, C, ncols, ld)`` with element (i, j) of
component c of the real (ri=0) / imaginary (ri=1) part at ``[ri, c, j, i]``.

Draw recipe (one numpy PCG64 generator per call, ``numpy.random.default_rng(seed)``):
  * leading components: uniform on [lo, hi) over an (m x ncols) row-major array, real
    part first, then imaginary part;
  * each lower component: c_k = c_{k-1} * 2^-53 * U(-1, 1), drawn in plane order
    re_c1, im_c1, re_c2, ...;
  * optional exact row scaling by 2^e_i, e_i integer.
The raw draws are not canonical (|c_1| may exceed half an ulp of c_0); the library and the
oracle each canonicalise their inputs with their own code.
"""
from __future__ import annotations

import numpy as np

__all__ = ["planes_from_complex", "uniform", "ones", "k_plus_ki", "householder_vectors",
           "geometric_sigma", "sample_entries", "row_exponents"]


def _empty(m: int, ncols: int, C: int, ld: int | None = None) -> np.ndarray:
    ld = m if ld is None else ld
    assert ld >= max(1, m)
    return np.zeros((2, C, ncols, ld), dtype=np.float64)


def planes_from_complex(Z: np.ndarray, C: int, ld: int | None = None) -> np.ndarray:
    """Exact double-valued complex matrix -> planes with zero lower components."""
    Z = np.asarray(Z)
    if Z.ndim == 1:
        Z = Z[:, None]
    m, ncols = Z.shape
    P = _empty(m, ncols, C, ld)
    P[0, 0, :, :m] = Z.real.T
    P[1, 0, :, :m] = Z.imag.T
    return P


def row_exponents(m: int, seed: int, lo: int = -20, hi: int = 20) -> np.ndarray:
    """Integer exponents e_i uniform in [lo, hi] (both ends included)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=m)


def uniform(m: int, ncols: int, C: int, seed: int, lo: float = -1.0, hi: float = 1.0,
            ld: int | None = None, row_exp: np.ndarray | None = None) -> np.ndarray:
    """Random complex multi-component matrix (see the module docstring for the recipe)."""
    rng = np.random.default_rng(seed)
    P = _empty(m, ncols, C, ld)
    re = rng.uniform(lo, hi, size=(m, ncols))
    im = rng.uniform(lo, hi, size=(m, ncols))
    comps = [(re, im)]
    for _ in range(1, C):
        pr, pi = comps[-1]
        r = pr * 2.0 ** -53 * rng.uniform(-1.0, 1.0, size=(m, ncols))
        i = pi * 2.0 ** -53 * rng.uniform(-1.0, 1.0, size=(m, ncols))
        comps.append((r, i))
    for c, (r, i) in enumerate(comps):
        if row_exp is not None:
            r = np.ldexp(r, row_exp[:, None])
            i = np.ldexp(i, row_exp[:, None])
        P[0, c, :, :m] = r.T
        P[1, c, :, :m] = i.T
    return P


def ones(n: int, nrhs: int, C: int) -> np.ndarray:
    """x_true = 1 + 0i in every entry."""
    P = _empty(n, nrhs, C)
    P[0, 0] = 1.0
    return P


def k_plus_ki(n: int, C: int) -> np.ndarray:
    """The paper's true solution x_k = k + k*i, k = 1..n (Sec. 4)."""
    P = _empty(n, 1, C)
    k = np.arange(1, n + 1, dtype=np.float64)
    P[0, 0, 0] = k
    P[1, 0, 0] = k
    return P


def householder_vectors(n: int, nrefl: int, seed: int):
    """Two sets of nrefl complex Gaussian vectors (exact doubles) for U and V."""
    rng = np.random.default_rng(seed)
    VL = rng.standard_normal((nrefl, n)) + 1j * rng.standard_normal((nrefl, n))
    VR = rng.standard_normal((nrefl, n)) + 1j * rng.standard_normal((nrefl, n))
    return VL, VR


def geometric_sigma(n: int, C: int, decades: float = 30.0) -> np.ndarray:
    """sigma_k = 10^(-decades*k/(n-1)), k = 0..n-1, as C greedy round-to-nearest
    binary64 components computed with mpmath at 400 bits.  Shape (n, C)."""
    import mpmath

    out = np.zeros((n, C))
    with mpmath.workprec(400):
        for k in range(n):
            x = mpmath.power(10, -mpmath.mpf(decades) * k / max(1, n - 1))
            for c in range(C):
                f = float(x)
                out[k, c] = f
                x = x - mpmath.mpf(f)
    return out


def sample_entries(n: int, count: int, seed: int):
    """count distinct (i, j) positions of an n x n matrix."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n * n, count, replace=False)
    return [(int(f // n), int(f % n)) for f in flat]
