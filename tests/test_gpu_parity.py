"""GPU parity against the CPU oracle, through the C ABI (libmplu.so via the binding).

Sizes here span several tiles / panels and a ragged tail while the oracle still finishes
in seconds.  Bounds:
  * products: |gpu - oracle| <= 4 (k+4) u (sum |a||b| + |c|) elementwise (cabs1 measure)
  * LU: identical pivots where the pivot gap is clear, factors within 100 n u
    (normwise), solutions within 10 n kappa u of the oracle's, backward error
    eta <= 10 n u from an exact residual
  * exactly representable factorisations: bit for bit on every path.
"""
import numpy as np
import pytest

import synthgen
from helpers import U_FMT, exact_lu_case, gemm_tol, pivot_gaps_clear, to_dev, to_host

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


@pytest.mark.parametrize("C", CS)
def test_renorm_matches_oracle_values(mp, orc, C):
    P = synthgen.uniform(77, 33, C, 1)
    T = to_dev(P)
    mp.renorm_(T)
    got = to_host(T)
    ref = orc.canon(P)
    d = orc.diff(got, ref)
    assert np.all(d == 0), "renormalised value changed"
    if C == 2:
        assert np.array_equal(got, ref)
    # non-overlap of consecutive components
    for c in range(C - 1):
        hi, lo = got[:, c], got[:, c + 1]
        assert np.all(np.abs(lo) <= np.spacing(np.abs(hi)) / 2)


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", ["3m", "4m"])
@pytest.mark.parametrize("ops", [("N", "N"), ("C", "N"), ("N", "C"), ("T", "T")])
def test_gemm_vs_oracle(mp, orc, C, method, ops):
    opA, opB = ops
    m, n, k = 70, 45, 37
    A = orc.canon(synthgen.uniform(m if opA == "N" else k, k if opA == "N" else m, C, 10))
    B = orc.canon(synthgen.uniform(k if opB == "N" else n, n if opB == "N" else k, C, 11))
    Cm = orc.canon(synthgen.uniform(m, n, C, 12))
    for alpha in (1, -1):
        ref = orc.gemm(A, B, Cm, method=3 if method == "3m" else 4, opA=opA, opB=opB,
                       alpha_sign=alpha)
        Td = to_dev(Cm)
        mp.gemm(to_dev(A), to_dev(B), Td, opA=opA, opB=opB, alpha=alpha, method=method)
        got = to_host(Td)
        d = orc.diff(got, ref)
        tol = gemm_tol(A, B, Cm, opA, opB, C, k)
        assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol)
    # beta = 0
    ref = orc.gemm(A, B, None, method=3 if method == "3m" else 4, opA=opA, opB=opB)
    got = to_host(mp.gemm(to_dev(A), to_dev(B), None, opA=opA, opB=opB, method=method))
    d = orc.diff(got, ref)
    tol = gemm_tol(A, B, None, opA, opB, C, k)
    assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol)


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", ["3m", "4m"])
def test_gemm_exact_on_dyadic_data(mp, C, method):
    rng = np.random.default_rng(5)
    m, n, k = 67, 41, 29
    Ac = (rng.integers(-99, 100, (m, k)) + 1j * rng.integers(-99, 100, (m, k))) / 8
    Bc = (rng.integers(-99, 100, (k, n)) + 1j * rng.integers(-99, 100, (k, n))) / 8
    Cc = (rng.integers(-99, 100, (m, n)) + 1j * rng.integers(-99, 100, (m, n))) / 8
    Td = to_dev(synthgen.planes_from_complex(Cc, C))
    mp.gemm(to_dev(synthgen.planes_from_complex(Ac, C)), to_dev(synthgen.planes_from_complex(Bc, C)),
            Td, alpha=-1, method=method)
    got = to_host(Td)
    assert np.array_equal((got[0, 0] + 1j * got[1, 0]).T, Cc - Ac @ Bc)
    assert not np.any(got[:, 1:])


@pytest.mark.parametrize("C", CS)
def test_gemm_real_data_3m_equals_4m_and_zero_imag(mp, orc, C):
    m, n, k = 40, 36, 50
    A = orc.canon(synthgen.uniform(m, k, C, 20))
    B = orc.canon(synthgen.uniform(k, n, C, 21))
    A[1] = 0
    B[1] = 0
    g3 = to_host(mp.gemm(to_dev(A), to_dev(B), None, method="3m"))
    g4 = to_host(mp.gemm(to_dev(A), to_dev(B), None, method="4m"))
    assert not np.any(g3[1])
    d = orc.diff(g3, g4)
    tol = gemm_tol(A, B, None, "N", "N", C, k)
    assert np.all(np.abs(d.real) <= tol)


def _lu_parity(mp, orc, C, n, panel, method, seed, m=None):
    m = n if m is None else m
    A = orc.canon(synthgen.uniform(m, n, C, seed))
    LUo, ipo, info_o = orc.getf2(A)
    T = to_dev(A)
    ipiv, info = mp.getrf(T, panel=panel, method=method)
    sync()
    LUg = to_host(T)
    ipg = ipiv.cpu().numpy()
    assert int(info.item()) == info_o == 0
    k_clear = pivot_gaps_clear(orc.hi_complex(LUo))
    assert np.array_equal(ipg[:k_clear], ipo[:k_clear])
    if k_clear == min(m, n):
        d = orc.diff(LUg, LUo)
        scale = np.abs(orc.hi_complex(LUo)).max()
        assert np.abs(d).max() <= 100 * max(m, n) * U_FMT[C] * scale
    return A, LUg, ipg, LUo, ipo


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", ["3m", "4m"])
def test_getrf_blocked_vs_oracle(mp, orc, C, method):
    _lu_parity(mp, orc, C, 200, 64, method, 30 + C)


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("n", [200, 203])
def test_getrf_strassen_vs_oracle(mp, orc, C, n):
    """The Strassen LU (Sec. 3, Table 1): trailing updates by one Winograd level over 3M
    (odd sizes peeled), the look-ahead's next-panel product in 3M; pivots and factors
    against the oracle, with and without the look-ahead."""
    _lu_parity(mp, orc, C, n, 64, "strassen", 50 + C)
    A = orc.canon(synthgen.uniform(n, n, C, 50 + C))
    LUo, ipo, _ = orc.getf2(A)
    T = to_dev(A)
    ipiv, info = mp.getrf(T, panel=64, method="strassen", lookahead=False)
    sync()
    assert int(info.item()) == 0
    k_clear = pivot_gaps_clear(orc.hi_complex(LUo))
    assert np.array_equal(ipiv.cpu().numpy()[:k_clear], ipo[:k_clear])
    if k_clear == n:
        d = orc.diff(to_host(T), LUo)
        assert np.abs(d).max() <= 100 * n * U_FMT[C] * np.abs(orc.hi_complex(LUo)).max()


@pytest.mark.parametrize("C", [2])
def test_getrf_unblocked_c1(mp, orc, C):
    """n = 64, panel = n (the unblocked "Normal LU"), 4M."""
    _lu_parity(mp, orc, C, 64, 64, "4m", 0)


@pytest.mark.parametrize("shape", [(150, 100), (100, 150), (257, 129)])
def test_getrf_rectangular(mp, orc, shape):
    m, n = shape
    _lu_parity(mp, orc, 2, n, 32, "3m", 40, m=m)


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("trans", ["N", "C"])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 6, 40])
def test_getrs_vs_oracle(mp, orc, C, trans, nrhs):
    """One-launch substitutions (up to 32 right-hand sides, in groups of 1, 2 or 4) and
    the blocked sweep (more), ragged last block row (n = 2 * 64 + 22)."""
    n = 150
    A = orc.canon(synthgen.uniform(n, n, C, 50 + C))
    B = orc.canon(synthgen.uniform(n, nrhs, C, 60 + C))
    LUo, ipo, _ = orc.getf2(A)
    Xo = orc.getrs(LUo, ipo, B, trans)
    T = to_dev(A)
    ipiv, info = mp.getrf(T, panel=64, method="3m")
    Bd = to_dev(B)
    mp.getrs(T, ipiv, Bd, trans=trans)
    Xg = to_host(Bd)
    kappa = float(np.real(np.linalg.cond(orc.hi_complex(A), np.inf)))
    d = orc.diff(Xg, Xo)
    assert np.abs(d).max() / np.abs(orc.hi_complex(Xo)).max() <= 10 * n * kappa * U_FMT[C]
    if trans == "C":
        AH = np.ascontiguousarray(np.transpose(A, (0, 1, 3, 2)))
        AH[1] *= -1
        eta = orc.backward_error(AH, Xg, B)
    else:
        eta = orc.backward_error(A, Xg, B)
    assert eta <= 10 * n * U_FMT[C]


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", ["3m", "4m"])
def test_exactly_representable_lu_bitwise(mp, C, method):
    for n, panel in ((64, 64), (150, 32)):
        A, L, U, ipiv_want = exact_lu_case(n, C, 7 + n)
        T = to_dev(A)
        ipiv, info = mp.getrf(T, panel=panel, method=method)
        sync()
        assert int(info.item()) == 0
        assert np.array_equal(ipiv.cpu().numpy(), ipiv_want)
        got = to_host(T)
        assert np.array_equal((got[0, 0] + 1j * got[1, 0]).T, np.tril(L, -1) + U)
        assert not np.any(got[:, 1:])
        xt = synthgen.planes_from_complex(np.arange(1, n + 1) * (1 + 1j), C)
        xc = (xt[0, 0] + 1j * xt[1, 0]).T
        Bd = to_dev(synthgen.planes_from_complex((A[0, 0] + 1j * A[1, 0]).T @ xc, C))
        mp.getrs(T, ipiv, Bd)
        assert np.array_equal(to_host(Bd), xt)


@pytest.mark.parametrize("C", [2, 4])
def test_zero_column_sets_info(mp, orc, C):
    n = 96
    A = orc.canon(synthgen.uniform(n, n, C, 70))
    A[:, :, 70, :] = 0.0
    _, _, info_o = orc.getf2(A)
    T = to_dev(A)
    _, info = mp.getrf(T, panel=32)
    sync()
    assert int(info.item()) == info_o == 71
    T = to_dev(np.zeros((2, C, 40, 40)))
    ipiv, info = mp.getrf(T, panel=16)
    sync()
    assert int(info.item()) == 1
    assert list(ipiv.cpu().numpy()) == list(range(1, 41))


@pytest.mark.parametrize("C", [2, 4])
@pytest.mark.parametrize("rows", [(3, 1), (150, 5), (7, 180)])
def test_pivot_tie_on_leading_component(mp, orc, C, rows):
    """Two candidates whose cabs1 agree in the leading component and differ below it:
    the larger full value wins whatever the row order, in one wave (3 vs 1) or across
    workgroups (150 vs 5, 7 vs 180)."""
    n = 200
    A = orc.canon(synthgen.uniform(n, n, C, 75))
    A[:, :, 0, :] *= 0.25  # column 0 otherwise below 0.5 in cabs1
    win, lose = rows
    A[:, :, 0, win] = 0.0
    A[:, :, 0, lose] = 0.0
    A[0, 0, 0, win] = 1.0
    A[0, 1, 0, win] = 2.0 ** -60
    A[0, 0, 0, lose] = 1.0
    A[0, 1, 0, lose] = -(2.0 ** -60)
    _, piv_o, _ = orc.getf2(A[:, :, :1, :].copy())
    assert int(piv_o[0]) == win + 1
    for method in ("3m", "split_i8"):
        T = to_dev(A)
        ipiv, info = mp.getrf(T, panel=64, method=method)
        sync()
        assert int(ipiv[0].item()) == win + 1


@pytest.mark.parametrize("C", [2, 4])
def test_nan_entries_finish_with_valid_pivots(mp, C):
    """NaN entries do not stop the factorisation or the solves: every pivot index stays
    within the rows still to be eliminated (ipiv[i] in [i + 1, n])."""
    n = 300
    A = synthgen.uniform(n, n, C, 76)
    A[0, 0, 5, 17] = np.nan       # one entry
    A[:, :, 130, :] = np.nan      # a whole column
    A[1, 0, 200, 40:90] = np.nan  # part of a column, imaginary parts
    for method in ("3m", "split_i8"):
        T = to_dev(A)
        ipiv, info = mp.getrf(T, panel=64, method=method)
        sync()
        piv = ipiv.cpu().numpy()
        assert np.all(piv >= np.arange(1, n + 1)) and np.all(piv <= n)
        B = to_dev(synthgen.uniform(n, 2, C, 77))
        mp.getrs(T, ipiv, B)
        sync()


def test_empty_and_tiny(mp, orc):
    import torch

    T = torch.zeros((2, 2, 0, 1), dtype=torch.float64, device="cuda")
    ipiv, info = mp.getrf(T, panel=64)
    sync()
    assert int(info.item()) == 0
    A = orc.canon(synthgen.uniform(1, 1, 2, 3))
    T = to_dev(A)
    ipiv, info = mp.getrf(T)
    sync()
    assert int(ipiv.item()) == 1 and np.array_equal(to_host(T), A)


@pytest.mark.parametrize("method", ["3m", "4m"])
def test_deterministic(mp, orc, method):
    A = orc.canon(synthgen.uniform(300, 300, 2, 80))
    outs = []
    for _ in range(2):
        T = to_dev(A)
        ipiv, info = mp.getrf(T, panel=64, method=method)
        sync()
        outs.append((to_host(T), ipiv.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


# ---------------------------------------------------------------- split (Ozaki) products
SPLIT = ["split_i8", "split_f64"]


def split_tol(A, B, Cm, opA, opB, C, k):
    """gemm_tol plus the slicing term k 2^-(53C+2) max_t|a_it| max_t|b_tj| (digits cover
    53C+2 bits below each row / column maximum)."""
    from helpers import cabs1_hi

    a = cabs1_hi(A)
    b = cabs1_hi(B)
    if opA != "N":
        a = a.T
    if opB != "N":
        b = b.T
    mx = np.outer(a.max(axis=1), b.max(axis=0))
    return gemm_tol(A, B, Cm, opA, opB, C, k) + 4 * k * 2.0 ** (-53 * C - 2) * mx * 4


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", SPLIT)
@pytest.mark.parametrize("ops", [("N", "N"), ("C", "T")])
def test_split_gemm_vs_oracle(mp, orc, C, method, ops):
    opA, opB = ops
    m, n, k = 70, 45, 150
    A = orc.canon(synthgen.uniform(m if opA == "N" else k, k if opA == "N" else m, C, 90))
    B = orc.canon(synthgen.uniform(k if opB == "N" else n, n if opB == "N" else k, C, 91))
    Cm = orc.canon(synthgen.uniform(m, n, C, 92))
    ref = orc.gemm(A, B, Cm, method=3, opA=opA, opB=opB, alpha_sign=-1)
    Td = to_dev(Cm)
    mp.gemm(to_dev(A), to_dev(B), Td, opA=opA, opB=opB, alpha=-1, method=method)
    d = orc.diff(to_host(Td), ref)
    tol = split_tol(A, B, Cm, opA, opB, C, k)
    assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol)


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", SPLIT)
def test_split_gemm_exact_on_dyadic_data(mp, C, method):
    """Pin P9: on small dyadic data every digit product is exact, so the split product
    equals the exact complex product bit for bit."""
    rng = np.random.default_rng(6)
    m, n, k = 67, 41, 130
    Ac = (rng.integers(-99, 100, (m, k)) + 1j * rng.integers(-99, 100, (m, k))) / 8
    Bc = (rng.integers(-99, 100, (k, n)) + 1j * rng.integers(-99, 100, (k, n))) / 8
    Cc = (rng.integers(-99, 100, (m, n)) + 1j * rng.integers(-99, 100, (m, n))) / 8
    Td = to_dev(synthgen.planes_from_complex(Cc, C))
    mp.gemm(to_dev(synthgen.planes_from_complex(Ac, C)), to_dev(synthgen.planes_from_complex(Bc, C)),
            Td, alpha=-1, method=method)
    got = to_host(Td)
    assert np.array_equal((got[0, 0] + 1j * got[1, 0]).T, Cc - Ac @ Bc)
    assert not np.any(got[:, 1:])


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", SPLIT)
def test_getrf_split_vs_oracle(mp, orc, C, method):
    A, LUg, ipg, LUo, ipo = _lu_parity(mp, orc, C, 200, 64, method, 35 + C)
    xt = synthgen.ones(200, 1, C)
    b = orc.matmul_exact(A, xt)
    Bd = to_dev(b)
    T = to_dev(LUg)
    mp.getrs(T, __import__("torch").from_numpy(ipg).cuda(), Bd)
    eta = orc.backward_error(A, to_host(Bd), b)
    assert eta <= 10 * 200 * U_FMT[C]


@pytest.mark.parametrize("S", [3, 4, 5, 6])
def test_split_f64_slice_count_sweep(mp, orc, S):
    """The division-count sweep of the paper's Ozaki LU (DD): fewer FP64 slices give a
    larger backward error; the default (6) meets the bound."""
    n = 160
    A = orc.canon(synthgen.uniform(n, n, 2, 44))
    b = orc.matmul_exact(A, synthgen.ones(n, 1, 2))
    T, Bd = to_dev(A), to_dev(b)
    mp.gesv(T, Bd, panel=32, method="split_f64", n_slices=S)
    sync()
    eta = orc.backward_error(A, to_host(Bd), b)
    if S == 6:
        assert eta <= 10 * n * U_FMT[2]
    else:
        assert eta < 1e-8


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("ncols", [1, 3, 16])
@pytest.mark.parametrize("opA", ["N", "C"])
def test_narrow_gemm_vs_oracle(mp, orc, C, ncols, opA):
    """Products with at most 16 output columns take the narrow kernel."""
    m, k = 150, 70
    A = orc.canon(synthgen.uniform(m if opA == "N" else k, k if opA == "N" else m, C, 95))
    B = orc.canon(synthgen.uniform(k, ncols, C, 96))
    Cm = orc.canon(synthgen.uniform(m, ncols, C, 97))
    ref = orc.gemm(A, B, Cm, method=4, opA=opA, alpha_sign=-1)
    Td = to_dev(Cm)
    mp.gemm(to_dev(A), to_dev(B), Td, opA=opA, alpha=-1, method="4m")
    d = orc.diff(to_host(Td), ref)
    tol = gemm_tol(A, B, Cm, opA, "N", C, k)
    assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol)


@pytest.mark.parametrize("C", [2, 4])
@pytest.mark.parametrize("panel", [96, 128])
def test_getrf_wide_panel_trsm_split(mp, orc, C, panel):
    """Panels whose triangle does not fit in LDS solve U12 in halves."""
    _lu_parity(mp, orc, C, 300, panel, "3m", 60 + C)


# ---------------------------------------------------------------- look-ahead schedule
@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", ["4m", "3m", "split_i8", "split_f64"])
@pytest.mark.parametrize("shape", [(300, 300), (333, 200), (200, 333)])
def test_lookahead_bitwise_equals_in_order(mp, orc, C, method, shape):
    """The two-stream look-ahead schedule performs the same operations on every element
    as the in-order one, so factors and pivots agree bit for bit (ragged last panel,
    tall and wide shapes)."""
    m, n = shape
    A = orc.canon(synthgen.uniform(m, n, C, 90 + C))
    outs = []
    for la in (False, True):
        T = to_dev(A)
        ipiv, info = mp.getrf(T, panel=64, method=method, m=m, lookahead=la)
        sync()
        outs.append((to_host(T), ipiv.cpu().numpy(), int(info.item())))
    assert outs[0][2] == outs[1][2] == 0
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][0], outs[1][0])


def test_lookahead_repeated_calls_and_gesv(mp, orc):
    """Back-to-back look-ahead factorisations reusing one workspace, then a solve on the
    caller's stream, all agree with the in-order schedule."""
    import torch

    n, C = 260, 2
    A = orc.canon(synthgen.uniform(n, n, C, 95))
    Bm = orc.canon(synthgen.uniform(n, 3, C, 96))
    ref = []
    T = to_dev(A)
    Bd = to_dev(Bm)
    mp.gesv(T, Bd, panel=32, method="3m", lookahead=False)
    sync()
    ref = (to_host(T), to_host(Bd))
    work = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    for _ in range(3):
        T = to_dev(A)
        Bd = to_dev(Bm)
        mp.gesv(T, Bd, panel=32, method="3m", work=work)
        sync()
        assert np.array_equal(to_host(T), ref[0]) and np.array_equal(to_host(Bd), ref[1])


def test_lookahead_two_streams_concurrently(mp, orc):
    """Two factorisations enqueued back to back on two different caller streams (each
    with its own second stream) run concurrently; each must still equal its in-order
    result."""
    import torch

    n, C = 300, 2
    A1 = orc.canon(synthgen.uniform(n, n, C, 101))
    A2 = orc.canon(synthgen.uniform(n, n, C, 102))
    ref = []
    for A in (A1, A2):
        T = to_dev(A)
        ipiv, _ = mp.getrf(T, panel=64, method="3m", lookahead=False)
        sync()
        ref.append((to_host(T), ipiv.cpu().numpy()))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    T1, T2 = to_dev(A1), to_dev(A2)
    sync()
    with torch.cuda.stream(s1):
        ip1, _ = mp.getrf(T1, panel=64, method="3m")
    with torch.cuda.stream(s2):
        ip2, _ = mp.getrf(T2, panel=64, method="3m")
    sync()
    for (R, rp), T, ip in zip(ref, (T1, T2), (ip1, ip2)):
        assert np.array_equal(ip.cpu().numpy(), rp)
        assert np.array_equal(to_host(T), R)


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", ["4m", "3m"] + SPLIT)
def test_matmul_uniform01_square_vs_oracle(mp, orc, C, method):
    """The matrix product of Sec. 2.4 (C := A B, square, leading components uniform on
    [0, 1]) in every product form, at a size with several K blocks and ragged tiles."""
    n = 150
    A = orc.canon(synthgen.uniform(n, n, C, 30, lo=0.0, hi=1.0))
    B = orc.canon(synthgen.uniform(n, n, C, 31, lo=0.0, hi=1.0))
    ref = orc.gemm(A, B, None, method=4 if method == "4m" else 3)
    got = to_host(mp.gemm(to_dev(A), to_dev(B), None, method=method))
    d = orc.diff(got, ref)
    tol = (split_tol if method in SPLIT else gemm_tol)(A, B, None, "N", "N", C, n)
    assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol)


def strassen_tol(A, B, Cm, C, k):
    """Normwise bound for one level of Winograd's variant over 3M products: the half-size
    operand sums are at most 3 max|a| (3 max|b|) in cabs1, each sub-product is accurate
    to 4 (k/2 + 4) u (k/2) times their maxima, and at most six matrix sums follow; every
    entry is within 64 (k + 4) u (k max|a| max|b| + |c|)."""
    from helpers import cabs1_hi

    t = 64 * (k + 4) * U_FMT[C] * k * cabs1_hi(A).max() * cabs1_hi(B).max()
    if Cm is not None:
        t = t + 64 * (k + 4) * U_FMT[C] * cabs1_hi(Cm)
    return t


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("shape", [(64, 64, 64), (150, 150, 150), (71, 45, 37), (1, 5, 3),
                                   (5, 1, 4), (33, 34, 1)])
def test_strassen_vs_oracle(mp, orc, C, shape):
    m, n, k = shape
    A = orc.canon(synthgen.uniform(m, k, C, 100))
    B = orc.canon(synthgen.uniform(k, n, C, 101))
    Cm = orc.canon(synthgen.uniform(m, n, C, 102))
    for alpha, use_c in ((1, False), (-1, True), (1, True)):
        ref = orc.gemm(A, B, Cm if use_c else None, method=3, alpha_sign=alpha)
        got = to_host(mp.gemm(to_dev(A), to_dev(B), to_dev(Cm) if use_c else None, alpha=alpha,
                              method="strassen"))
        d = orc.diff(got, ref)
        tol = strassen_tol(A, B, Cm if use_c else None, C, k)
        assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol)


@pytest.mark.parametrize("C", CS)
def test_strassen_exact_on_dyadic_data(mp, C):
    """On small dyadic data every matrix sum and product of the Winograd schedule is exact,
    so the result equals the exact product bit for bit (a wrong block, sign or peeling
    step would show as an error of the size of the entries)."""
    rng = np.random.default_rng(8)
    for (m, n, k) in ((67, 41, 130), (64, 64, 65), (2, 2, 2)):
        Ac = (rng.integers(-99, 100, (m, k)) + 1j * rng.integers(-99, 100, (m, k))) / 8
        Bc = (rng.integers(-99, 100, (k, n)) + 1j * rng.integers(-99, 100, (k, n))) / 8
        Cc = (rng.integers(-99, 100, (m, n)) + 1j * rng.integers(-99, 100, (m, n))) / 8
        Td = to_dev(synthgen.planes_from_complex(Cc, C))
        mp.gemm(to_dev(synthgen.planes_from_complex(Ac, C)),
                to_dev(synthgen.planes_from_complex(Bc, C)), Td, alpha=-1, method="strassen")
        got = to_host(Td)
        assert np.array_equal((got[0, 0] + 1j * got[1, 0]).T, Cc - Ac @ Bc)
        assert not np.any(got[:, 1:])


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("method", ["3m", "4m"])
def test_long_product_independent_of_tiling(mp, orc, C, method):
    """Products deeper than 128 re-level their accumulators at the same steps of k in
    every kernel: a block of a large product (32 x 32 tiles) equals the same block computed
    alone (16 x 16 tiles, and for 4M with few columns the narrow kernel) bit for bit."""
    import torch

    m = n = 720   # 23 x 23 = 529 tiles of 32 x 32: the large-product kernel
    k = 300
    A = orc.canon(synthgen.uniform(m, k, C, 110))
    B = orc.canon(synthgen.uniform(k, n, C, 111))
    Cm = orc.canon(synthgen.uniform(m, n, C, 112))
    Ad, Bd = to_dev(A), to_dev(B)
    big = to_host(mp.gemm(Ad, Bd, to_dev(Cm), alpha=-1, method=method))
    for (r0, c0, mr, nc) in ((37, 101, 90, 70), (500, 3, 64, 12), (0, 700, 720, 20)):
        As = torch.from_numpy(np.ascontiguousarray(A[:, :, :, r0:r0 + mr])).cuda()
        Bs = torch.from_numpy(np.ascontiguousarray(B[:, :, c0:c0 + nc, :])).cuda()
        Cs = torch.from_numpy(np.ascontiguousarray(Cm[:, :, c0:c0 + nc, r0:r0 + mr])).cuda()
        small = to_host(mp.gemm(As, Bs, Cs, alpha=-1, method=method))
        assert np.array_equal(small, big[:, :, c0:c0 + nc, r0:r0 + mr])


@pytest.mark.parametrize("C", CS)
@pytest.mark.parametrize("k", [37, 64, 100])
def test_trailing_depth_product_independent_of_tiling(mp, orc, C, k):
    """At trailing-update depths (k <= 128) the double-double 3M and real products sum
    their cross products a_hi b_lo + a_lo b_hi on the FP64 matrix cores in the same 4-deep
    steps in both tilings: a block of a large product (32 x 32 tiles) equals the same
    block computed alone (16 x 16 tiles) bit for bit, for every format, also for depths
    that are not a multiple of the staging depths (the tilings pad the last 4-deep steps
    with different numbers of zero steps), and in the real product."""
    import torch

    m = n = 720   # 23 x 23 = 529 tiles of 32 x 32: the large-product kernel
    A = orc.canon(synthgen.uniform(m, k, C, 130))
    B = orc.canon(synthgen.uniform(k, n, C, 131))
    Cm = orc.canon(synthgen.uniform(m, n, C, 132))
    big = to_host(mp.gemm(to_dev(A), to_dev(B), to_dev(Cm), alpha=-1, method="3m"))
    bigr = to_host(mp.dgemm(to_dev(A[0]), to_dev(B[0]), to_dev(Cm[0]), alpha=-1))
    for (r0, c0, mr, nc) in ((37, 101, 90, 70), (500, 3, 64, 12), (0, 700, 720, 20)):
        As = np.ascontiguousarray(A[:, :, :, r0:r0 + mr])
        Bs = np.ascontiguousarray(B[:, :, c0:c0 + nc, :])
        Cs = np.ascontiguousarray(Cm[:, :, c0:c0 + nc, r0:r0 + mr])
        small = to_host(mp.gemm(torch.from_numpy(As).cuda(), torch.from_numpy(Bs).cuda(),
                                torch.from_numpy(Cs).cuda(), alpha=-1, method="3m"))
        assert np.array_equal(small, big[:, :, c0:c0 + nc, r0:r0 + mr])
        smallr = to_host(mp.dgemm(torch.from_numpy(np.ascontiguousarray(As[0])).cuda(),
                                  torch.from_numpy(np.ascontiguousarray(Bs[0])).cuda(),
                                  torch.from_numpy(np.ascontiguousarray(Cs[0])).cuda(), alpha=-1))
        assert np.array_equal(smallr, bigr[:, c0:c0 + nc, r0:r0 + mr])
    # the real product is the real part of the complex 3M product on real data
    def embed(R):
        Z = np.zeros((2,) + R.shape)
        Z[0] = R
        return Z
    z = to_host(mp.gemm(to_dev(embed(A[0])), to_dev(embed(B[0])), to_dev(embed(Cm[0])),
                        alpha=-1, method="3m"))
    assert np.array_equal(z[0], bigr)
    assert not np.any(z[1])


def test_solve_api_and_singular_check(mp, orc):
    """lu_factor / lu_solve leave their inputs alone and agree with gesv; solve with
    check_errors raises on an exactly singular matrix with and without autograd."""
    import torch

    n, C = 70, 2
    A = orc.canon(synthgen.uniform(n, n, C, 120))
    B = orc.canon(synthgen.uniform(n, 3, C, 121))
    Ad, Bd = to_dev(A), to_dev(B)
    LU, piv, info = mp.lu_factor(Ad)
    X = mp.lu_solve(LU, piv, Bd)
    XH = mp.lu_solve(LU, piv, Bd, adjoint=True)
    assert np.array_equal(to_host(Ad), A) and np.array_equal(to_host(Bd), B)
    A2, B2 = to_dev(A), to_dev(B)
    mp.gesv(A2, B2)
    assert np.array_equal(to_host(X), to_host(B2))
    LUo, ipo, _ = orc.getf2(A)
    XHo = orc.getrs(LUo, ipo, B, "C")
    kappa = float(np.real(np.linalg.cond(orc.hi_complex(A), np.inf)))
    d = orc.diff(to_host(XH), XHo)
    assert np.abs(d).max() / np.abs(orc.hi_complex(XHo)).max() <= 10 * n * kappa * U_FMT[C]
    assert np.array_equal(to_host(mp.solve(Ad, Bd, check_errors=True)), to_host(X))
    S = A.copy()
    S[:, :, 5, :] = 0.0
    for grad in (False, True):
        Sd = to_dev(S).requires_grad_(grad)
        with pytest.raises(torch.linalg.LinAlgError):
            mp.solve(Sd, to_dev(B), check_errors=True)


def test_strassen_empty_and_k0(mp, orc):
    """Degenerate Strassen-Winograd products: m = 0 leaves nothing to do; k = 0 gives
    beta C (here C itself with beta = 1, zeros with beta = 0)."""
    import torch

    C = 2
    Cm = orc.canon(synthgen.uniform(6, 4, C, 130))
    A = torch.zeros((2, C, 0, 6), dtype=torch.float64, device="cuda")
    B = torch.zeros((2, C, 4, 0), dtype=torch.float64, device="cuda")
    got = to_host(mp.gemm(A, B, to_dev(Cm), k=0, method="strassen"))
    assert np.array_equal(got, Cm)
    got0 = to_host(mp.gemm(A, B, None, k=0, method="strassen"))
    assert not np.any(got0)
    E = torch.zeros((2, C, 3, 0), dtype=torch.float64, device="cuda")
    F = torch.zeros((2, C, 0, 3), dtype=torch.float64, device="cuda")
    assert mp.gemm(E, F, None, m=0, method="strassen").numel() == 0


@pytest.mark.parametrize("lookahead", [False, True])
def test_expired_waits_report_timeout(mp, orc, lookahead):
    """The panel's bounded waits, forced expired from the host (MPLU_FLAG_EXPIRE_WAITS),
    give up and every kernel ends: the call completes with info = MPLU_INFO_SYNC_TIMEOUT.
    The next ordinary call on the same workspace is unaffected (bit for bit the
    reference factorisation)."""
    import ctypes as ct

    import torch

    n, C = 300, 2
    A = orc.canon(synthgen.uniform(n, n, C, 120))
    T = to_dev(A)
    ref_ip, ref_info = mp.getrf(T, panel=64, method="3m", lookahead=False)
    sync()
    ref = to_host(T)
    o = mp._opts(64, "3m", lookahead=lookahead, flags=mp.FLAG_EXPIRE_WAITS)
    nb = ct.c_size_t()
    assert mp.lib().mplu_zgetrf_wsbytes(C, n, n, ct.byref(o), ct.byref(nb)) == 0
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    T = to_dev(A)
    rc = mp.lib().mplu_zgetrf(C, n, n, mp._zmat(T), ipiv.data_ptr(), info.data_ptr(),
                              ct.byref(o), work.data_ptr(), work.numel(), mp._stream())
    assert rc == 0
    sync()
    assert int(info.item()) == -9999
    T = to_dev(A)
    ipiv2, info2 = mp.getrf(T, panel=64, method="3m", lookahead=lookahead, work=work)
    sync()
    assert int(info2.item()) == 0
    assert np.array_equal(ipiv2.cpu().numpy(), ref_ip.cpu().numpy())
    assert np.array_equal(to_host(T), ref)
