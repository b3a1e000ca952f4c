"""Pins for the oracle's LU, solves, products and residual against facts that do not come
from the oracle itself: exact rational elimination, exactly representable factorisations,
mpmath solves at 1024 bits, LAPACK's pivot choice, and the backward-error invariant."""
from fractions import Fraction

import numpy as np
import pytest

import synthgen

CS = [2, 3, 4]
U_FMT = {2: 2.0 ** -104, 3: 2.0 ** -157, 4: 2.0 ** -209}


def fr(v):
    return sum((Fraction(float(c)) for c in v), Fraction(0))


def elem(P, i, j):
    C = P.shape[1]
    return fr(P[0, :C, j, i]), fr(P[1, :C, j, i])


def zmul(a, b):
    return a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0]


def zdiv(a, b):
    d = b[0] * b[0] + b[1] * b[1]
    return (a[0] * b[0] + a[1] * b[1]) / d, (a[1] * b[0] - a[0] * b[1]) / d


def zsub(a, b):
    return a[0] - b[0], a[1] - b[1]


def cabs1(a):
    return abs(a[0]) + abs(a[1])


def to_frac_matrix(P, m=None, n=None):
    m = P.shape[3] if m is None else m
    n = P.shape[2] if n is None else n
    return [[elem(P, i, j) for j in range(n)] for i in range(m)]


def exact_gepp(M):
    """Rational Gaussian elimination with partial pivoting by cabs1, ties -> lowest row.
    Returns (ipiv 1-based, factors, relative cabs1 gap of each pivot choice)."""
    M = [row[:] for row in M]
    n = len(M)
    ipiv, gaps = [], []
    for k in range(n):
        vals = [cabs1(M[i][k]) for i in range(k, n)]
        best = max(vals)
        p = k + vals.index(best)
        rest = sorted(vals, reverse=True)
        gaps.append(float((rest[0] - rest[1]) / rest[0]) if len(rest) > 1 and rest[0] else 1.0)
        ipiv.append(p + 1)
        M[k], M[p] = M[p], M[k]
        if best == 0:
            continue
        for i in range(k + 1, n):
            M[i][k] = zdiv(M[i][k], M[k][k])
            for j in range(k + 1, n):
                M[i][j] = zsub(M[i][j], zmul(M[i][k], M[k][j]))
    return ipiv, M, gaps


def exact_solve(M, b):
    ipiv, F, _ = exact_gepp(M)
    n = len(M)
    x = list(b)
    for k in range(n):
        p = ipiv[k] - 1
        x[k], x[p] = x[p], x[k]
    for i in range(n):
        for k in range(i):
            x[i] = zsub(x[i], zmul(F[i][k], x[k]))
    for i in reversed(range(n)):
        for k in range(i + 1, n):
            x[i] = zsub(x[i], zmul(F[i][k], x[k]))
        x[i] = zdiv(x[i], F[i][i])
    return x


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("real", [False, True])
def test_tiny_lu_matches_exact_elimination(orc, C, real):
    """Pin P2: n <= 6 random inputs.  The pivot sequence equals exact rational GEPP
    whenever every exact cabs1 gap exceeds 2^-90, PA - LU is within the rounding bound,
    and the solution is within 10 n kappa u of the exact solution.  With zero imaginary
    parts (the oracle of the real routines) the factors stay real and the same holds
    against real rational elimination."""
    u = U_FMT[C]
    checked = 0
    for seed in range(12):
        n = 2 + seed % 5
        A = orc.canon(synthgen.uniform(n, n, C, 100 + seed))
        if real:
            A[1] = 0.0
        M = to_frac_matrix(A)
        ipiv_x, F_x, gaps = exact_gepp(M)
        LU, ipiv, info = orc.getf2(A)
        assert info == 0
        if real:
            assert not np.any(LU[1])
        if min(gaps) > 2.0 ** -90:
            assert list(ipiv) == ipiv_x
            checked += 1
        # backward error of the factors: P A = L U + E, |E| <= 8 (n+2) u |L||U|
        F = to_frac_matrix(LU)
        PA = [row[:] for row in M]
        for k in range(n):
            p = ipiv[k] - 1
            PA[k], PA[p] = PA[p], PA[k]
        for i in range(n):
            for j in range(n):
                s = (Fraction(0), Fraction(0))
                mag = Fraction(0)
                for t in range(min(i, j) + 1):
                    lv = (Fraction(1), Fraction(0)) if t == i else F[i][t]
                    uv = F[t][j]
                    s = (s[0] + zmul(lv, uv)[0], s[1] + zmul(lv, uv)[1])
                    mag += Fraction(abs(complex(float(lv[0]), float(lv[1]))) *
                                    abs(complex(float(uv[0]), float(uv[1]))))
                err = abs(complex(float(s[0] - PA[i][j][0]), float(s[1] - PA[i][j][1])))
                assert err <= 8 * (n + 2) * u * float(mag) * 1.01
        # solution vs the exact one
        xt = synthgen.ones(n, 1, C)
        b = orc.matmul_exact(A, xt)
        x = orc.getrs(LU, ipiv, b)
        bx = [elem(b, i, 0) for i in range(n)]
        xs = exact_solve(M, bx)
        Ah = orc.hi_complex(A)
        kappa = np.linalg.cond(Ah, np.inf)
        num = max(abs(complex(float(elem(x, i, 0)[0] - xs[i][0]),
                              float(elem(x, i, 0)[1] - xs[i][1]))) for i in range(n))
        den = max(abs(complex(float(v[0]), float(v[1]))) for v in xs)
        assert num / den <= 10 * n * kappa * u
    assert checked >= 8


def exact_lu_case(n, C, seed, ld=None):
    """A = P^T L U with dyadic entries chosen so that every intermediate value of the
    elimination is exact in binary64: |Re l|, |Im l| <= 1/4 (so cabs1(l) <= 1/2 and the
    true pivot always wins), U's diagonal in {+-2^e, +-i 2^e, (+-1+-i) 2^e} (exact
    reciprocals), all entries multiples of 2^-8."""
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
    LU = L @ U                      # exact: |entries| small, 16 fractional bits
    A = np.zeros_like(LU)
    A[perm] = LU                    # row i of L U sits at row perm[i] of A
    # expected LAPACK-style pivots: simulate the row swaps of the elimination
    pos = list(perm)                # pos[i] = current row of the row holding (LU)_i
    at = {pos[i]: i for i in range(n)}
    ipiv = []
    for k in range(n):
        p = pos[k]
        ipiv.append(p + 1)
        other = at[k]
        at[k], at[p] = k, other
        pos[k], pos[other] = k, p
    return synthgen.planes_from_complex(A, C, ld), L, U, np.array(ipiv, dtype=np.int32)


@pytest.mark.parametrize("C", CS)
def test_exactly_representable_lu_bitwise(orc, C):
    """Pin P3: an exactly representable factorisation is reproduced bit for bit."""
    for seed in range(3):
        n = 24 + 7 * seed
        A, L, U, ipiv_want = exact_lu_case(n, C, 200 + seed)
        LU, ipiv, info = orc.getf2(A)
        assert info == 0
        assert np.array_equal(ipiv, ipiv_want)
        got = orc.hi_complex(LU)
        want = np.tril(L, -1) + U
        assert np.array_equal(got, want)
        assert not np.any(LU[:, 1:])          # lower components stay exactly zero
        # solve: x exact too
        xt = synthgen.planes_from_complex(np.arange(1, n + 1) * (1 + 1j), C)
        b = orc.matmul_exact(A, xt)
        x = orc.getrs(LU, ipiv, b)
        assert np.array_equal(x, xt)


@pytest.mark.parametrize("C", CS)
def test_solve_vs_mpmath_1024_bits(orc, C):
    """Pin P5: oracle solve vs mpmath.lu_solve at 1024 bits (library routine)."""
    import mpmath

    n = 20
    A = orc.canon(synthgen.uniform(n, n, C, 300 + C))
    xt = synthgen.ones(n, 1, C)
    b = orc.matmul_exact(A, xt)
    x, LU, ipiv, info = orc.gesv(A, b)
    with mpmath.workprec(1024):
        Am = mpmath.matrix(n, n)
        bm = mpmath.matrix(n, 1)
        for i in range(n):
            for j in range(n):
                re = sum(mpmath.mpf(float(v)) for v in A[0, :, j, i])
                im = sum(mpmath.mpf(float(v)) for v in A[1, :, j, i])
                Am[i, j] = mpmath.mpc(re, im)
            bm[i] = mpmath.mpc(sum(mpmath.mpf(float(v)) for v in b[0, :, 0, i]),
                               sum(mpmath.mpf(float(v)) for v in b[1, :, 0, i]))
        xm = mpmath.lu_solve(Am, bm)
        errs, mags = [], []
        for i in range(n):
            xr = sum(mpmath.mpf(float(v)) for v in x[0, :, 0, i])
            xi = sum(mpmath.mpf(float(v)) for v in x[1, :, 0, i])
            errs.append(float(abs(mpmath.mpc(xr, xi) - xm[i])))
            mags.append(float(abs(xm[i])))
    kappa = float(np.real(np.linalg.cond(orc.hi_complex(A), np.inf)))
    assert max(errs) / max(mags) <= 10 * n * kappa * U_FMT[C]


def test_pivots_match_lapack_when_gaps_are_clear(orc):
    """Pin P6: LAPACK zgetrf (torch.linalg.lu_factor on the leading components, same
    cabs1 measure) picks the same pivots wherever its own cabs1 gap is clear."""
    import torch

    n = 64
    for seed in range(3):
        A = orc.canon(synthgen.uniform(n, n, 2, 400 + seed))
        Ah = torch.from_numpy(orc.hi_complex(A))
        LUd, piv = torch.linalg.lu_factor(Ah)
        LUd = LUd.numpy()
        piv = piv.numpy()
        _, ipiv, _ = orc.getf2(A)
        for k in range(n - 1):
            ukk = LUd[k, k]
            c_piv = abs(ukk.real) + abs(ukk.imag)
            others = [abs((LUd[i, k] * ukk).real) + abs((LUd[i, k] * ukk).imag)
                      for i in range(k + 1, n)]
            if max(others) > c_piv * (1 - 1e-9):
                break
            assert piv[k] == ipiv[k], (seed, k)
        else:
            k = n
        assert k >= n // 2


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("trans", ["N", "C"])
def test_backward_error_invariant(orc, C, trans):
    """Pin P7: eta = ||b - A x|| / (||A|| ||x||) <= 10 n u with an exact residual."""
    n = 48
    A = orc.canon(synthgen.uniform(n, n, C, 500 + C))
    B = orc.canon(synthgen.uniform(n, 3, C, 501 + C))
    LU, ipiv, info = orc.getf2(A)
    X = orc.getrs(LU, ipiv, B, trans)
    if trans == "C":
        AH = np.ascontiguousarray(np.transpose(A, (0, 1, 3, 2)))
        AH[1] *= -1
        eta = orc.backward_error(AH, X, B)
    else:
        eta = orc.backward_error(A, X, B)
    assert eta <= 10 * n * U_FMT[C]
    assert eta > 0


@pytest.mark.parametrize("C", CS)
def test_singular_column_sets_info(orc, C):
    n = 10
    A = orc.canon(synthgen.uniform(n, n, C, 600))
    A[:, :, 3, :] = 0.0                      # column 3 exactly zero
    _, _, info = orc.getf2(A)
    assert info == 4
    A = np.zeros((2, C, n, n))
    _, ipiv, info = orc.getf2(A)
    assert info == 1 and list(ipiv) == list(range(1, n + 1))


def test_residual_is_exact(orc):
    """The residual routine returns RN(b - A x) of the exact value."""
    n, C = 5, 3
    A = orc.canon(synthgen.uniform(n, n, C, 700))
    X = orc.canon(synthgen.uniform(n, 2, C, 701))
    B = orc.canon(synthgen.uniform(n, 2, C, 702))
    r = orc.resid(A, X, B)
    for i in range(n):
        for k in range(2):
            s = elem(B, i, k)
            for j in range(n):
                s = zsub(s, zmul(elem(A, i, j), elem(X, j, k)))
            assert r[i, k].real == float(s[0]) and r[i, k].imag == float(s[1])


@pytest.mark.parametrize("C", CS)
def test_gemm_exact_on_dyadic_data(orc, C):
    """On small dyadic integers every product and sum is exact: 3M and 4M must both
    equal the exact complex product (numpy complex128 is exact here)."""
    rng = np.random.default_rng(800 + C)
    m, n, k = 7, 9, 11
    Ac = (rng.integers(-99, 100, (m, k)) + 1j * rng.integers(-99, 100, (m, k))) / 8
    Bc = (rng.integers(-99, 100, (k, n)) + 1j * rng.integers(-99, 100, (k, n))) / 8
    Cc = (rng.integers(-99, 100, (m, n)) + 1j * rng.integers(-99, 100, (m, n))) / 8
    A = synthgen.planes_from_complex(Ac, C)
    B = synthgen.planes_from_complex(Bc, C)
    Cm = synthgen.planes_from_complex(Cc, C)
    for method in (3, 4):
        out = orc.gemm(A, B, Cm, method=method, alpha_sign=-1)
        assert np.array_equal(orc.hi_complex(out), Cc - Ac @ Bc)
        out = orc.gemm(A, B, None, method=method)
        assert np.array_equal(orc.hi_complex(out), Ac @ Bc)


@pytest.mark.parametrize("C", CS)
def test_gemm_4m_is_rounded_exact_product_and_3m_bound(orc, C):
    """4M: each part within 2^-(53C) of the exact product.  3M vs 4M:
    |C3 - C4| <= 2 (K+4) u (|ReA|+|ImA|)(|ReB|+|ImB|) (Higham 1992 form)."""
    m, n, k = 5, 4, 13
    A = orc.canon(synthgen.uniform(m, k, C, 900 + C))
    B = orc.canon(synthgen.uniform(k, n, C, 910 + C))
    c4 = orc.gemm(A, B, None, method=4)
    c3 = orc.gemm(A, B, None, method=3)
    u = U_FMT[C]
    for i in range(m):
        for j in range(n):
            ex = (Fraction(0), Fraction(0))
            bound = 0.0
            for t in range(k):
                p = zmul(elem(A, i, t), elem(B, t, j))
                ex = (ex[0] + p[0], ex[1] + p[1])
                a, b = orc.hi_complex(A)[i, t], orc.hi_complex(B)[t, j]
                bound += (abs(a.real) + abs(a.imag)) * (abs(b.real) + abs(b.imag))
            g4 = elem(c4, i, j)
            g3 = elem(c3, i, j)
            for part in (0, 1):
                assert abs(g4[part] - ex[part]) <= abs(ex[part]) * Fraction(2) ** (-53 * C)
                assert float(abs(g3[part] - g4[part])) <= 2 * (k + 4) * u * bound


@pytest.mark.parametrize("C", CS)
def test_gemm_real_inputs_3m_equals_4m(orc, C):
    """Im(A) = Im(B) = 0: the 3M imaginary part is exactly 0 and the real parts agree."""
    m, n, k = 6, 5, 17
    A = orc.canon(synthgen.uniform(m, k, C, 1000 + C))
    B = orc.canon(synthgen.uniform(k, n, C, 1010 + C))
    A[1] = 0.0
    B[1] = 0.0
    c4 = orc.gemm(A, B, None, method=4)
    c3 = orc.gemm(A, B, None, method=3)
    assert np.array_equal(c3, c4)
    assert not np.any(c3[1])


@pytest.mark.parametrize("C", [2])
def test_gemm_transpose_modes(orc, C):
    m, n, k = 4, 6, 5
    A = orc.canon(synthgen.uniform(k, m, C, 1100))   # stored k x m, used as op(A) = A^T / A^H
    B = orc.canon(synthgen.uniform(n, k, C, 1101))   # stored n x k, used as op(B)
    AT = np.ascontiguousarray(np.transpose(A, (0, 1, 3, 2)))
    BT = np.ascontiguousarray(np.transpose(B, (0, 1, 3, 2)))
    for method in (3, 4):
        ref = orc.gemm(AT, BT, None, method=method)
        assert np.array_equal(orc.gemm(A, B, None, method=method, opA="T", opB="T"), ref)
        AH, BH = AT.copy(), BT.copy()
        AH[1] *= -1
        BH[1] *= -1
        ref = orc.gemm(AH, BH, None, method=method)
        assert np.array_equal(orc.gemm(A, B, None, method=method, opA="C", opB="C"), ref)
