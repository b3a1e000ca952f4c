"""Pins for the oracle's auxiliary routines, each against a fact that does not come from
the oracle: exact rationals, an independent high-precision construction, singular values,
closed-form derivatives and exactly known norms.

  diff          every GPU-vs-oracle elementwise comparison goes through it
  round_to      format conversion (greedy round-to-nearest of the exact value)
  gen_illcond   the ill-conditioned matrix U diag(sigma) V^H of the TD / QD configuration
  solve_grad    the gradient of a loss through x = A^-1 b (g_b = A^-H g_x, g_A = -g_b x^H)
  cond_inf_est  the condition estimate used by the forward-error bounds 10 n kappa u
"""
from fractions import Fraction

import numpy as np
import pytest

import synthgen

CS = [2, 3, 4]
U_FMT = {2: 2.0 ** -104, 3: 2.0 ** -157, 4: 2.0 ** -209}


def fr(v):
    return sum((Fraction(float(c)) for c in v), Fraction(0))


def greedy(x: Fraction, C: int):
    out = []
    for _ in range(C):
        if x == 0 or abs(x) < Fraction(2) ** -1022:
            out.append(0.0)
            x = Fraction(0)
            continue
        f = float(x)
        out.append(f)
        x -= Fraction(f)
    return out


def raw_components(rng, C, e0=None):
    """C components with random signs, exponent gaps and zeros; not necessarily canonical
    (gaps of 40..60 bits let neighbouring components overlap)."""
    e = int(rng.integers(-40, 40)) if e0 is None else e0
    out = [float(np.ldexp(rng.uniform(0.5, 1.0) * rng.choice([-1, 1]), e))]
    for _ in range(1, C):
        e -= int(rng.integers(40, 61))
        out.append(0.0 if rng.random() < 0.1 else float(np.ldexp(rng.uniform(-1, 1), e)))
    return out


# ------------------------------------------------------------------------------- diff
def _pair_planes(xs, ys, CX, CY):
    """Lists of (re, im) component lists -> two (2, C, 1, m) plane arrays."""
    m = len(xs)
    X = np.zeros((2, CX, 1, m))
    Y = np.zeros((2, CY, 1, m))
    for i in range(m):
        for ri in range(2):
            X[ri, :, 0, i] = xs[i][ri]
            Y[ri, :, 0, i] = ys[i][ri]
    return X, Y


@pytest.mark.parametrize("CX", CS)
@pytest.mark.parametrize("CY", CS)
def test_diff_is_rounded_exact_difference(orc, CX, CY):
    """diff(X, Y) = RN(X - Y) of the exact values, bit for bit, for every pair of formats.
    Most cases make Y agree with X in its leading components, so that the difference lives
    in the lower components only: a comparator that looked at fewer components than given
    would return 0 or a wrong value there."""
    rng = np.random.default_rng(1000 + 10 * CX + CY)
    xs, ys = [], []
    for t in range(400):
        x = [raw_components(rng, CX), raw_components(rng, CX)]
        kind = t % 4
        if kind in (0, 1):
            # Y = X rounded to CY components, plus a perturbation far below the leading
            # component (kind 1: none, so the difference is X's tail beyond CY components)
            y = []
            for ri in range(2):
                v = fr(x[ri])
                if kind == 0:
                    v += Fraction(float(np.ldexp(rng.uniform(-1, 1), -80 - int(rng.integers(0, 60)))))
                y.append(greedy(v, CY))
        elif kind == 2:
            y = [[-c for c in x[0]][:CY] + [0.0] * max(0, CY - CX),
                 raw_components(rng, CY)]
        else:
            y = [raw_components(rng, CY), raw_components(rng, CY)]
        xs.append(x)
        ys.append([list(y[0][:CY]) + [0.0] * (CY - len(y[0][:CY])),
                   list(y[1][:CY]) + [0.0] * (CY - len(y[1][:CY]))])
    X, Y = _pair_planes(xs, ys, CX, CY)
    D = orc.diff(X, Y)
    assert D.shape == (len(xs), 1)
    lower_only = 0
    for i in range(len(xs)):
        for ri, got in ((0, D[i, 0].real), (1, D[i, 0].imag)):
            exact = fr(X[ri, :, 0, i]) - fr(Y[ri, :, 0, i])
            ref = float(exact) if abs(exact) >= Fraction(2) ** -1022 or exact == 0 else None
            if ref is None:
                continue
            assert got == ref and np.signbit(got) == np.signbit(ref) or (got == 0 and ref == 0), \
                (CX, CY, i, ri, got, ref)
            if X[ri, 0, 0, i] == Y[ri, 0, 0, i] and exact != 0:
                lower_only += 1
    assert lower_only > 50   # the leading components alone would decide nothing there


def test_diff_geometry_and_sign(orc):
    """Shape (rows, cols), column-major planes with ld > rows, and the sign of X - Y."""
    C, m, n, ld = 2, 3, 4, 5
    X = np.zeros((2, C, n, ld))
    Y = np.zeros((2, C, n, ld))
    for j in range(n):
        for i in range(m):
            X[0, 0, j, i] = 1.0 + i
            X[0, 1, j, i] = 2.0 ** -60 * (j + 1)     # the difference is the lower part
            Y[0, 0, j, i] = 1.0 + i
            Y[1, 0, j, i] = -(i + 10 * j)
    D = orc.diff(X, Y, m=m)
    assert D.shape == (m, n)
    for j in range(n):
        for i in range(m):
            assert D[i, j].real == 2.0 ** -60 * (j + 1)
            assert D[i, j].imag == i + 10 * j
    D2 = orc.diff(Y, X, m=m)
    assert np.array_equal(D2, -D)


# ----------------------------------------------------------------------------- round_to
@pytest.mark.parametrize("Cin", CS)
@pytest.mark.parametrize("Cout", CS)
def test_round_to_is_greedy_rounding_of_exact_value(orc, Cin, Cout):
    """round_to gives c0 = RN(x), c1 = RN(x - c0), ... of the exact sum of the input
    components (non-canonical inputs included), bit for bit, in both parts."""
    rng = np.random.default_rng(2000 + 10 * Cin + Cout)
    m, n = 7, 9
    P = np.zeros((2, Cin, n, m))
    for j in range(n):
        for i in range(m):
            for ri in range(2):
                P[ri, :, j, i] = raw_components(rng, Cin)
    P[:, :, 0, 0] = 0.0                                  # zero element
    P[0, :, 1, 1] = [(-1) ** c * 2.0 ** (-60 * c) for c in range(Cin)]  # alternating signs
    Q = orc.round_to(P, Cout)
    assert Q.shape == (2, Cout, n, m)
    for j in range(n):
        for i in range(m):
            for ri in range(2):
                ref = greedy(fr(P[ri, :, j, i]), Cout)
                assert [float(v).hex() for v in Q[ri, :, j, i]] == [v.hex() for v in ref], \
                    (Cin, Cout, i, j, ri)


# -------------------------------------------------------------------------- gen_illcond
def _mp_reflector_product(V, n, mpmath, reverse=False):
    """Product of the reflectors H_t = I - tau v_t v_t^H, tau = 2 / (v^H v), in index
    order (reverse: descending index), in mpmath at the working precision."""
    P = mpmath.eye(n)
    order = range(V.shape[0] - 1, -1, -1) if reverse else range(V.shape[0])
    for t in order:
        v = mpmath.matrix([mpmath.mpc(float(z.real), float(z.imag)) for z in V[t]])
        vh = v.H
        tau = 2 / (vh * v)[0]
        H = mpmath.eye(n) - tau * (v * vh)
        P = P * H
    return P


@pytest.mark.parametrize("C", [3, 4])
def test_gen_illcond_matches_svd_construction(orc, C):
    """A = U diag(sigma) V^H with U = H_0 H_1 ... (left reflectors in index order) and
    V^H = H'_{r-1} ... H'_0 (right reflectors in descending order), every reflector
    H = I - tau v v^H unitary.  Rebuilt here in mpmath at 600 bits from the same vectors:
    elementwise agreement within the rounding of 2 r reflector applications, and the
    singular values of the oracle's matrix equal sigma (1 down to 1e-30) to far better
    than the smallest one -- a generator that ignored sigma, dropped a reflector or
    conjugated the wrong side fails one of the two."""
    import mpmath

    n, nrefl = 6, 3
    sig = synthgen.geometric_sigma(n, C)
    VL, VR = synthgen.householder_vectors(n, nrefl, 77 + C)
    A = orc.gen_illcond(n, C, sig, VL, VR)
    Ah = orc.hi_complex(A)
    assert np.abs(Ah - np.diag(np.diag(Ah))).max() > 1e-2     # really mixed
    with mpmath.workprec(600):
        U = _mp_reflector_product(VL, n, mpmath)
        VH = _mp_reflector_product(VR, n, mpmath, reverse=True)
        S = mpmath.zeros(n, n)
        for k in range(n):
            S[k, k] = sum(mpmath.mpf(float(c)) for c in sig[k])
        Aref = U * S * VH
        Am = mpmath.matrix(n, n)
        worst = mpmath.mpf(0)
        for i in range(n):
            for j in range(n):
                re = sum(mpmath.mpf(float(c)) for c in A[0, :, j, i])
                im = sum(mpmath.mpf(float(c)) for c in A[1, :, j, i])
                Am[i, j] = mpmath.mpc(re, im)
                worst = max(worst, abs(Am[i, j] - Aref[i, j]))
        assert float(worst) <= 10 * nrefl * n * U_FMT[C]
        sv = mpmath.svd_c(Am, compute_uv=False)
        sv = sorted([sv[k] for k in range(n)], reverse=True)
        for k in range(n):
            want = sum(mpmath.mpf(float(c)) for c in sig[k])
            assert abs(sv[k] - want) <= 100 * nrefl * n * U_FMT[C], (k, sv[k], want)
        assert float(sv[0] / sv[-1]) == pytest.approx(1e30, rel=1e-12)


# --------------------------------------------------------------------------- gradient
def _fr_matrix(P, rows, cols):
    return [[(fr(P[0, :, j, i]), fr(P[1, :, j, i])) for j in range(cols)] for i in range(rows)]


def _zmul(a, b):
    return a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0]


def _zdiv(a, b):
    d = b[0] * b[0] + b[1] * b[1]
    return (a[0] * b[0] + a[1] * b[1]) / d, (a[1] * b[0] - a[0] * b[1]) / d


def _exact_solve(M, B):
    """Exact rational solve M X = B (Gauss-Jordan, any nonzero pivot)."""
    n, r = len(M), len(B[0])
    T = [list(M[i]) + list(B[i]) for i in range(n)]
    for k in range(n):
        p = next(i for i in range(k, n) if T[i][k] != (0, 0))
        T[k], T[p] = T[p], T[k]
        piv = T[k][k]
        T[k] = [_zdiv(v, piv) for v in T[k]]
        for i in range(n):
            if i != k and T[i][k] != (0, 0):
                f = T[i][k]
                T[i] = [(v[0] - w[0], v[1] - w[1])
                        for v, w in zip(T[i], [_zmul(f, u) for u in T[k]])]
    return [row[n:] for row in T]


def _zabs(a):
    return float(abs(complex(float(a[0]), float(a[1]))))


@pytest.mark.parametrize("C", CS)
def test_solve_grad_matches_exact_derivative(orc, C):
    """For L = Re sum(conj(c) x), x = A^-1 b, the exact gradients are g_b = A^-H c and
    g_A = -g_b x^H (rational arithmetic on the same inputs).  The oracle's gradient must
    agree within the forward-error bound of its solves, 10 n kappa u, elementwise relative
    to the largest entry: a sign error, a missing conjugation or a solve with A instead of
    A^H is an O(1) difference."""
    n, nrhs = 4, 2
    A = orc.canon(synthgen.uniform(n, n, C, 3000 + C))
    B = orc.canon(synthgen.uniform(n, nrhs, C, 3100 + C))
    Gx = orc.canon(synthgen.uniform(n, nrhs, C, 3200 + C))
    X, LU, ipiv, info = orc.gesv(A, B)
    assert info == 0
    Gb, GA = orc.solve_grad(LU, ipiv, X, Gx)
    Am = _fr_matrix(A, n, n)
    AH = [[(Am[j][i][0], -Am[j][i][1]) for j in range(n)] for i in range(n)]
    Bm = _fr_matrix(B, n, nrhs)
    Gm = _fr_matrix(Gx, n, nrhs)
    Xs = _exact_solve(Am, Bm)
    Gbs = _exact_solve(AH, Gm)
    kappa = float(np.real(np.linalg.cond(orc.hi_complex(A), np.inf)))
    tol = 10 * n * kappa * U_FMT[C]
    mb = max(_zabs(v) for row in Gbs for v in row)
    for i in range(n):
        for r in range(nrhs):
            got = (fr(Gb[0, :, r, i]), fr(Gb[1, :, r, i]))
            d = (got[0] - Gbs[i][r][0], got[1] - Gbs[i][r][1])
            assert _zabs(d) <= tol * mb, (i, r)
    GAs = [[None] * n for _ in range(n)]
    ma = 0.0
    for i in range(n):
        for j in range(n):
            s = (Fraction(0), Fraction(0))
            for r in range(nrhs):
                xc = (Xs[j][r][0], -Xs[j][r][1])
                p = _zmul(Gbs[i][r], xc)
                s = (s[0] - p[0], s[1] - p[1])
            GAs[i][j] = s
            ma = max(ma, _zabs(s))
    for i in range(n):
        for j in range(n):
            got = (fr(GA[0, :, j, i]), fr(GA[1, :, j, i]))
            d = (got[0] - GAs[i][j][0], got[1] - GAs[i][j][1])
            assert _zabs(d) <= 2 * tol * ma, (i, j)


@pytest.mark.parametrize("C", [2])
def test_solve_grad_directional_derivative(orc, C):
    """The gradient predicts the change of L = Re sum(conj(c) x) along a direction
    (E, e) of (A, b): dL = Re<g_A, E> + Re<g_b, e>, checked against a central difference
    of exact rational solves (the loss is a rational function, so the step only sets a
    truncation term of order h^2)."""
    n, nrhs = 3, 2
    A = orc.canon(synthgen.uniform(n, n, C, 3300))
    B = orc.canon(synthgen.uniform(n, nrhs, C, 3301))
    Gx = orc.canon(synthgen.uniform(n, nrhs, C, 3302))
    E = synthgen.uniform(n, n, 1, 3303)[:, 0]
    e = synthgen.uniform(n, nrhs, 1, 3304)[:, 0]
    X, LU, ipiv, _ = orc.gesv(A, B)
    Gb, GA = orc.solve_grad(LU, ipiv, X, Gx)
    Am, Bm, cm = _fr_matrix(A, n, n), _fr_matrix(B, n, nrhs), _fr_matrix(Gx, n, nrhs)
    h = Fraction(1, 2 ** 40)

    def loss(t):
        At = [[(Am[i][j][0] + t * Fraction(float(E[0, j, i])), Am[i][j][1] + t * Fraction(float(E[1, j, i])))
               for j in range(n)] for i in range(n)]
        Bt = [[(Bm[i][r][0] + t * Fraction(float(e[0, r, i])), Bm[i][r][1] + t * Fraction(float(e[1, r, i])))
               for r in range(nrhs)] for i in range(n)]
        Xt = _exact_solve(At, Bt)
        return sum(cm[i][r][0] * Xt[i][r][0] + cm[i][r][1] * Xt[i][r][1]
                   for i in range(n) for r in range(nrhs))

    fd = float((loss(h) - loss(-h)) / (2 * h))
    pred = 0.0
    for i in range(n):
        for j in range(n):
            pred += GA[0, 0, j, i] * E[0, j, i] + GA[1, 0, j, i] * E[1, j, i]
        for r in range(nrhs):
            pred += Gb[0, 0, r, i] * e[0, r, i] + Gb[1, 0, r, i] * e[1, r, i]
    assert abs(pred - fd) <= 1e-9 * max(1.0, abs(fd))


# -------------------------------------------------------------------- condition estimate
def test_inv_norm_estimate_exact_on_diagonal(orc):
    """||diag(d)^-1||_1 = max 1/|d_i|, found exactly by the estimator."""
    n, C = 9, 2
    d = np.array([3.0, -0.5 + 0.25j, 1j, 2.0, 0.125, 4 + 4j, -1.0, 0.75j, 8.0])
    A = synthgen.planes_from_complex(np.diag(d), C)
    LU, ipiv, _ = orc.getf2(A)
    for tr in ("N", "C"):
        est = orc.inv_norm1_est(LU, ipiv, tr)
        assert est == pytest.approx(float(np.max(1 / np.abs(d))), rel=1e-14)


@pytest.mark.parametrize("C", [2, 4])
def test_cond_estimate_against_explicit_inverse(orc, C):
    """On small matrices whose inverse double precision computes accurately, the
    estimate of kappa_inf is a lower bound of the true value and at least a third of it;
    with rows scaled over 2^+-8 the 1- and inf-norms of the inverse differ, so an
    estimator of the wrong one (solves with A instead of A^H) is caught."""
    rng_exp = synthgen.row_exponents(16, 41, -8, 8)
    hits = 0
    for seed in range(6):
        n = 16
        A = orc.canon(synthgen.uniform(n, n, C, 4000 + seed, row_exp=rng_exp))
        LU, ipiv, _ = orc.getf2(A)
        Ah = orc.hi_complex(A)
        Ai = np.linalg.inv(Ah)
        true_inf = float(np.abs(Ah).sum(axis=1).max() * np.abs(Ai).sum(axis=1).max())
        true_one = float(np.abs(Ah).sum(axis=1).max() * np.abs(Ai).sum(axis=0).max())
        est = orc.cond_inf_est(A, LU, ipiv)
        assert est <= true_inf * (1 + 1e-10)
        assert est >= true_inf / 3
        hits += abs(est - true_inf) <= 1e-10 * true_inf
        if abs(true_one - true_inf) > 0.2 * true_inf:
            assert abs(est - true_one) > 1e-3 * true_one or abs(est - true_inf) < 1e-10 * true_inf
    assert hits >= 4
