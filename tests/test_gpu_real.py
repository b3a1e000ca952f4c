"""Real matrices (the Im = 0 case of the method): mplu_dgetrf / dgetrs / dgesv / dgemm
through the C ABI.

The oracle for a real matrix is the complex oracle on the same matrix with zero imaginary
parts (its exact-then-round 4M arithmetic then reduces to real arithmetic, and its
reciprocal to conj(b)/|b|^2 = b/b^2).  Checks:
  * dgemm against the oracle's product, elementwise within 4 (k + 4) u sum |a||b|, and
    bitwise equal to the real part of the complex 3M product on the embedded operands;
  * dgetrf against the oracle (pivots where the gap is clear, factors within
    100 n u), its look-ahead schedule bitwise equal to the in-order one;
  * dgesv / dgetrs ('N' and 'T') against the oracle: pivots where the gap is clear,
    solutions within 10 n kappa u, backward error within 10 n u (exact residual);
  * exactly representable real factorisations bit for bit; a zero column sets info;
  * the full-size real DD solve at n = 4096 within 10 n u.
"""
import numpy as np
import pytest

import synthgen
from helpers import U_FMT, gemm_tol, pivot_gaps_clear

pytestmark = pytest.mark.gpu

CS = [2, 3, 4]


@pytest.fixture(scope="module")
def mp():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_16013_amd as m

    m.lib()
    return m


def sync():
    import torch

    torch.cuda.synchronize()


def dev(P):
    import torch

    return torch.from_numpy(np.ascontiguousarray(P)).to("cuda")


def host(T):
    return T.detach().cpu().numpy().copy()


def real_planes(m, ncols, C, seed, orc):
    """Canonical real planes (C, ncols, m): the real part of a canonical complex draw."""
    return np.ascontiguousarray(orc.canon(synthgen.uniform(m, ncols, C, seed))[0])


def embed(R):
    """Real planes (C, ncols, ld) -> complex planes (2, C, ncols, ld), imaginary part 0."""
    Z = np.zeros((2,) + R.shape)
    Z[0] = R
    return Z


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("ops", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_dgemm_vs_oracle_and_complex_3m(mp, orc, C, ops):
    opA, opB = ops
    m, n, k = 70, 45, 150
    A = real_planes(m if opA == "N" else k, k if opA == "N" else m, C, 10, orc)
    B = real_planes(k if opB == "N" else n, n if opB == "N" else k, C, 11, orc)
    Cm = real_planes(m, n, C, 12, orc)
    zop = {"N": "N", "T": "T"}
    for alpha, use_c in ((1, True), (-1, True), (1, False)):
        ref = orc.gemm(embed(A), embed(B), embed(Cm) if use_c else None, method=4,
                       opA=zop[opA], opB=zop[opB], alpha_sign=alpha)
        got = host(mp.dgemm(dev(A), dev(B), dev(Cm) if use_c else None, opA=opA, opB=opB,
                            alpha=alpha))
        d = orc.diff(embed(got), ref)
        tol = gemm_tol(embed(A), embed(B), embed(Cm) if use_c else None, opA, opB, C, k)
        assert np.all(np.abs(d.real) <= tol) and not np.any(d.imag)
        # the real product is the real part of the complex 3M product, bit for bit
        Zc = dev(embed(Cm)) if use_c else None
        z = host(mp.gemm(dev(embed(A)), dev(embed(B)), Zc, opA=opA, opB=opB, alpha=alpha,
                         method="3m"))
        assert np.array_equal(z[0], got)
        assert not np.any(z[1])


def test_dgemm_exact_on_dyadic_data(mp):
    rng = np.random.default_rng(3)
    m, n, k = 67, 41, 200
    for C in CS:
        A = rng.integers(-99, 100, (m, k)) / 8
        B = rng.integers(-99, 100, (k, n)) / 8
        Cc = rng.integers(-99, 100, (m, n)) / 8
        P = lambda X: synthgen.planes_from_complex(X.astype(complex), C)[0]
        got = host(mp.dgemm(dev(P(A)), dev(P(B)), dev(P(Cc)), alpha=-1))
        assert np.array_equal(got[0].T, Cc - A @ B)
        assert not np.any(got[1:])


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("shape", [(200, 200, 64), (150, 100, 32), (100, 150, 32),
                                   (260, 260, 128), (257, 200, 96)])
def test_dgetrf_vs_oracle_and_schedules(mp, orc, C, shape):
    """The real factorisation against the oracle (pivots where the gap is clear, factors
    within 100 max(m, n) u), and the look-ahead schedule bitwise equal to the in-order one."""
    m, n, panel = shape
    A = real_planes(m, n, C, 30 + C, orc)
    T = dev(A)
    ipiv, info = mp.dgetrf(T, panel=panel)
    T2 = dev(A)
    ipiv2, info2 = mp.dgetrf(T2, panel=panel, lookahead=False)
    sync()
    assert int(info.item()) == int(info2.item()) == 0
    assert np.array_equal(ipiv.cpu().numpy(), ipiv2.cpu().numpy())
    LUg = host(T)
    assert np.array_equal(LUg, host(T2))
    LUo, ipo, info_o = orc.getf2(embed(A))
    assert info_o == 0 and not np.any(LUo[1])
    k_clear = pivot_gaps_clear(orc.hi_complex(LUo))
    assert np.array_equal(ipiv.cpu().numpy()[:k_clear], ipo[:k_clear])
    if k_clear == min(m, n):
        d = orc.diff(embed(LUg), LUo)
        scale = np.abs(orc.hi_complex(LUo)).max()
        assert np.abs(d).max() <= 100 * max(m, n) * U_FMT[C] * scale


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("nrhs", [1, 3, 40])
def test_dgesv_dgetrs_vs_oracle(mp, orc, C, trans, nrhs):
    n = 150
    A = real_planes(n, n, C, 50 + C, orc)
    B = real_planes(n, nrhs, C, 60 + C, orc)
    LUo, ipo, info_o = orc.getf2(embed(A))
    assert info_o == 0
    assert not np.any(LUo[1])
    Xo = orc.getrs(LUo, ipo, embed(B), "N" if trans == "N" else "C")
    if trans == "N":
        Ad, Bd = dev(A), dev(B)
        ipiv, info = mp.dgesv(Ad, Bd, panel=64)
        sync()
        assert int(info.item()) == 0
        LUg = host(Ad)
    else:
        Ad = dev(A)
        ipiv, info = mp.dgetrf(Ad, panel=64)
        Bd = dev(B)
        mp.dgetrs(Ad, ipiv, Bd, trans="T")
        sync()
        LUg = host(Ad)
    k_clear = pivot_gaps_clear(orc.hi_complex(LUo))
    assert np.array_equal(ipiv.cpu().numpy()[:k_clear], ipo[:k_clear])
    if k_clear == n:
        d = orc.diff(embed(LUg), LUo)
        assert np.abs(d).max() <= 100 * n * U_FMT[C] * np.abs(orc.hi_complex(LUo)).max()
    Xg = embed(host(Bd))
    kappa = float(np.linalg.cond(A[0].T, np.inf))
    d = orc.diff(Xg, Xo)
    assert np.abs(d).max() / np.abs(orc.hi_complex(Xo)).max() <= 10 * n * kappa * U_FMT[C]
    Aop = embed(A) if trans == "N" else embed(np.ascontiguousarray(np.transpose(A, (0, 2, 1))))
    assert orc.backward_error(Aop, Xg, embed(B)) <= 10 * n * U_FMT[C]


@pytest.mark.parametrize("C", CS)
def test_real_exactly_representable_lu_bitwise(mp, C):
    """A = P^T L U with dyadic L (|l| <= 1/4), dyadic U and power-of-two diagonal: every
    intermediate is exact in binary64, so factors, pivots and the solution are exact."""
    for n, panel in ((64, 64), (150, 32)):
        rng = np.random.default_rng(70 + n)
        L = np.eye(n) + np.tril(rng.integers(-64, 65, (n, n)) / 256.0, -1)
        U = np.triu(rng.integers(-256, 257, (n, n)) / 256.0, 1)
        U[np.diag_indices(n)] = 2.0 ** rng.integers(-2, 3, n) * rng.choice([-1, 1], n)
        perm = rng.permutation(n)
        A = np.zeros((n, n))
        A[perm] = L @ U
        pos, at, want = list(perm), {p: i for i, p in enumerate(perm)}, []
        for k in range(n):
            p = pos[k]
            want.append(p + 1)
            other = at[k]
            at[k], at[p] = k, other
            pos[k], pos[other] = k, p
        P = lambda X: synthgen.planes_from_complex(np.asarray(X, dtype=complex), C)[0]
        x = np.arange(1, n + 1, dtype=float)
        Ad, Bd = dev(P(A)), dev(P(A @ x))
        ipiv, info = mp.dgesv(Ad, Bd, panel=panel)
        sync()
        assert int(info.item()) == 0
        assert np.array_equal(ipiv.cpu().numpy(), np.array(want, dtype=np.int32))
        got = host(Ad)
        assert np.array_equal(got[0].T, np.tril(L, -1) + U)
        assert not np.any(got[1:])
        assert np.array_equal(host(Bd), P(x))


def test_real_zero_column_sets_info(mp, orc):
    n, C = 100, 2
    A = real_planes(n, n, C, 80, orc)
    A[:, 37, :] = 0.0
    Ad = dev(A)
    _, info = mp.dgetrf(Ad, panel=32)
    sync()
    _, _, info_o = orc.getf2(embed(A))
    assert int(info.item()) == info_o == 38


def test_real_dd_n4096_backward_error(mp, orc):
    """The full size of the complex headline, real DD, panel 64: exact residual."""
    n, C = 4096, 2
    A = real_planes(n, n, C, 0, orc)
    b = orc.matmul_exact(embed(A), synthgen.ones(n, 1, C))
    Ad, Bd = dev(A), dev(b[0])
    _, info = mp.dgesv(Ad, Bd, panel=64)
    sync()
    assert int(info.item()) == 0
    eta = orc.backward_error(embed(A), embed(host(Bd)), b)
    assert eta <= 10 * n * U_FMT[C], eta


def test_real_empty_and_tiny(mp, orc):
    import torch

    # n = 0: nothing to do, info 0
    A0 = torch.zeros((2, 0, 1), dtype=torch.float64, device="cuda")
    B0 = torch.zeros((2, 1, 1), dtype=torch.float64, device="cuda")
    _, info = mp.dgesv(A0, B0[:, :0, :0].contiguous())
    assert int(info.item()) == 0
    # 1 x 1: x = b / a
    for C in CS:
        A = real_planes(1, 1, C, 90 + C, orc)
        B = real_planes(1, 1, C, 95 + C, orc)
        Ad, Bd = dev(A), dev(B)
        ipiv, info = mp.dgesv(Ad, Bd)
        sync()
        assert int(info.item()) == 0 and int(ipiv.item()) == 1
        Xo = orc.getrs(*orc.getf2(embed(A))[:2], embed(B))
        d = orc.diff(embed(host(Bd)), Xo)
        assert np.abs(d).max() <= 8 * U_FMT[C] * np.abs(orc.hi_complex(Xo)).max()


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", ["split_i8", "split_f64"])
def test_real_split_lu_vs_oracle(mp, orc, C, method):
    """The split trailing update on real operands: solution and backward error against
    the oracle, the look-ahead schedule bitwise equal to the in-order one, and exact
    dyadic factorisations bit for bit."""
    n = 200
    A = real_planes(n, n, C, 140 + C, orc)
    B = real_planes(n, 2, C, 150 + C, orc)
    LUo, ipo, _ = orc.getf2(embed(A))
    Xo = orc.getrs(LUo, ipo, embed(B))
    Ad, Bd = dev(A), dev(B)
    ipiv, info = mp.dgesv(Ad, Bd, panel=64, method=method)
    A2 = dev(A)
    ipiv2, _ = mp.dgetrf(A2, panel=64, method=method, lookahead=False)
    sync()
    assert int(info.item()) == 0
    assert np.array_equal(host(Ad), host(A2))
    assert np.array_equal(ipiv.cpu().numpy(), ipiv2.cpu().numpy())
    Xg = embed(host(Bd))
    kappa = float(np.linalg.cond(A[0].T, np.inf))
    d = orc.diff(Xg, Xo)
    assert np.abs(d).max() / np.abs(orc.hi_complex(Xo)).max() <= 10 * n * kappa * U_FMT[C]
    assert orc.backward_error(embed(A), Xg, embed(B)) <= 10 * n * U_FMT[C]
    # exactly representable: L dyadic with |l| <= 1/4, U dyadic, power-of-two diagonal
    rng = np.random.default_rng(160 + C)
    m = 150
    L = np.eye(m) + np.tril(rng.integers(-64, 65, (m, m)) / 256.0, -1)
    U = np.triu(rng.integers(-256, 257, (m, m)) / 256.0, 1)
    U[np.diag_indices(m)] = 2.0 ** rng.integers(-2, 3, m) * rng.choice([-1, 1], m)
    P = lambda X: synthgen.planes_from_complex(np.asarray(X, dtype=complex), C)[0]
    Ed = dev(P(L @ U))
    _, info = mp.dgetrf(Ed, panel=32, method=method)
    sync()
    assert int(info.item()) == 0
    assert np.array_equal(host(Ed)[0].T, np.tril(L, -1) + U)
