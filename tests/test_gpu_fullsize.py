"""Full-size checks of the factorisation's pieces at the shapes the benchmark runs.

  * backward error of every format and trailing-update form at n = 4096 (panels 64 and
    128), each from the oracle's exact residual;
  * the trailing-update product itself at its real shape (m = n = 4032 or 3968, depth
    64 or 128: thousands of 32 x 32 tiles, no re-levelling), a sampled 24 x 24 block of
    A22 - L21 U12 elementwise against the oracle's product of the same rows and columns;
  * the adjoint of x = A^-1 b against the oracle's gradient (g_b = A^-H g_x by the
    oracle's getrs('C'), g_A = -g_b x^H), elementwise.
"""
import numpy as np
import pytest

import synthgen
from helpers import U_FMT, to_dev, to_host

pytestmark = pytest.mark.gpu


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


_SYSTEMS = {}


def system_n4096(orc, C):
    """A uniform[-1,1] (lower components scaled by 2^-53 U(-1,1)), b = A 1 exactly."""
    if C not in _SYSTEMS:
        _SYSTEMS.clear()
        n = 4096
        A = orc.canon(synthgen.uniform(n, n, C, 0))
        b = orc.matmul_exact(A, synthgen.ones(n, 1, C))
        _SYSTEMS[C] = (A, b)
    return _SYSTEMS[C]


GRID = [(C, meth, K) for C in (2, 3, 4)
        for meth, K in (("3m", 64), ("3m", 128), ("4m", 64), ("split_i8", 64),
                        ("split_i8", 128), ("split_f64", 64), ("strassen", 64))]


@pytest.mark.parametrize("C,method,panel", GRID)
def test_eta_n4096_every_form(mp, orc, C, method, panel):
    """eta = ||b - A x|| / (||A|| ||x||) <= 10 n u by the oracle's exact residual, for
    DD / TD / QD and the 3M, 4M, both split and the Strassen-Winograd trailing updates
    (Sec. 3, Table 1's comparison of LU forms)."""
    import torch

    n = 4096
    A, b = system_n4096(orc, C)
    T, x = to_dev(A), to_dev(b)
    ipiv, info = mp.gesv(T, x, panel=panel, method=method)
    sync()
    assert int(info.item()) == 0
    xh = to_host(x)
    del T, x
    torch.cuda.empty_cache()
    eta = orc.backward_error(A, xh, b)
    print(f"C={C} {method} K={panel}: eta={eta:.3e} (bound {10 * n * U_FMT[C]:.3e})")
    assert eta <= 10 * n * U_FMT[C]


@pytest.mark.parametrize("C", [2, 3, 4])
@pytest.mark.parametrize("k", [64, 128])
def test_trailing_update_shape_sampled(mp, orc, C, k):
    """A22 := A22 - L21 U12 at the first trailing update of n = 4096 (m = n = 4096 - k),
    the launch the factorisation spends most of its time in, in every product form:
    24 sampled rows x 24 sampled columns elementwise against the oracle's product of the
    same rows and columns, within 4 (k + 4) u (sum |l||u| + |a|) (plus the slicing term
    2^-(53C+2) below each row / column maximum for the split forms)."""
    import torch

    m = 4096 - k
    L = orc.canon(synthgen.uniform(m, k, C, 21))
    U = orc.canon(synthgen.uniform(k, m, C, 22))
    A22 = orc.canon(synthgen.uniform(m, m, C, 23))
    rng = np.random.default_rng(4)
    rows = np.sort(rng.choice(m, 24, replace=False))
    rows[-1] = m - 1                           # the ragged last tile row
    cols = np.sort(rng.choice(m, 24, replace=False))
    cols[0] = 0
    Ls = np.ascontiguousarray(L[:, :, :, rows])
    Us = np.ascontiguousarray(U[:, :, cols, :])
    As = np.ascontiguousarray(A22[:, :, cols][:, :, :, rows])
    a = (np.abs(Ls[0, 0]) + np.abs(Ls[1, 0])).T
    u = (np.abs(Us[0, 0]) + np.abs(Us[1, 0])).T
    S = a @ u + (np.abs(As[0, 0]) + np.abs(As[1, 0])).T
    slicing = 16 * k * 2.0 ** (-53 * C - 2) * np.outer(
        (np.abs(L[0, 0]) + np.abs(L[1, 0])).T.max(axis=1)[rows],
        (np.abs(U[0, 0]) + np.abs(U[1, 0])).T.max(axis=0)[cols])
    Ld, Ud = to_dev(L), to_dev(U)
    worst = {}
    for method in ("3m", "4m", "split_i8", "split_f64"):
        ref = orc.gemm(Ls, Us, As, method=4 if method == "4m" else 3, alpha_sign=-1)
        Td = to_dev(A22)
        mp.gemm(Ld, Ud, Td, alpha=-1, method=method)
        got = to_host(Td[:, :, cols][:, :, :, rows])
        del Td
        d = orc.diff(np.ascontiguousarray(got), ref)
        tol = 4 * (k + 4) * U_FMT[C] * S + (slicing if method.startswith("split") else 0)
        assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol), method
        worst[method] = float(np.max(np.abs(d) / S))
    print(f"C={C} k={k} m={m}: err / sum|l||u| {worst}")
    del Ld, Ud
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,nrhs", [(256, 16), (203, 5)])
def test_adjoint_vs_oracle_gradient(mp, orc, n, nrhs):
    """MPSolve.backward (getrs('C') on the saved factors, then the rank-nrhs update)
    against the oracle's gradient from its own factors: g_b within 10 n kappa u of the
    oracle's (both solve A^H g_b = g_x), g_A = -g_b x^H within 20 n kappa u normwise."""
    C = 2
    A = orc.canon(synthgen.uniform(n, n, C, 30))
    B = orc.canon(synthgen.uniform(n, nrhs, C, 31))
    c = orc.canon(synthgen.uniform(n, nrhs, C, 32))
    Xo, LUo, ipo, info = orc.gesv(A, B)
    assert info == 0
    gbo, gAo = orc.solve_grad(LUo, ipo, Xo, c)
    kappa = orc.cond_inf_est(A, LUo, ipo)
    Ad = to_dev(A).requires_grad_(True)
    Bd = to_dev(B).requires_grad_(True)
    X = mp.solve(Ad, Bd)
    X.backward(to_dev(c))
    sync()
    gA, gB = to_host(Ad.grad), to_host(Bd.grad)
    u = U_FMT[C]
    eb = np.abs(orc.diff(gB, gbo)).max() / np.abs(orc.hi_complex(gbo)).max()
    eA = np.abs(orc.diff(gA, gAo)).max() / np.abs(orc.hi_complex(gAo)).max()
    print(f"n={n} nrhs={nrhs} kappa={kappa:.2e}: g_b {eb:.2e}, g_A {eA:.2e}")
    assert eb <= 10 * n * kappa * u
    assert eA <= 20 * n * kappa * u


@pytest.mark.parametrize("C,k", [(4, 5248 + 203), (2, 9920 + 77)])
def test_deep_split_i8_product_in_pieces(mp, orc, C, k):
    """INT8 split products deeper than the INT32 limit of a combined level sum (three
    times 64 S 65^2 per 64-deep chunk below 2^31: k = 5 248 for QD, 9 920 for DD) run as
    consecutive pieces accumulated into the result: elementwise against the oracle within
    the product bound, the slicing term and one rounding of the running sum per piece."""
    m, n = 37, 29
    A = orc.canon(synthgen.uniform(m, k, C, 40))
    B = orc.canon(synthgen.uniform(k, n, C, 41))
    Cm = orc.canon(synthgen.uniform(m, n, C, 42))
    ref = orc.gemm(A, B, Cm, method=3, alpha_sign=-1)
    Td = to_dev(Cm)
    mp.gemm(to_dev(A), to_dev(B), Td, alpha=-1, method="split_i8")
    got = to_host(Td)
    a = (np.abs(A[0, 0]) + np.abs(A[1, 0])).T
    b = (np.abs(B[0, 0]) + np.abs(B[1, 0])).T
    S = a @ b + (np.abs(Cm[0, 0]) + np.abs(Cm[1, 0])).T
    slicing = 16 * k * 2.0 ** (-53 * C - 2) * np.outer(a.max(axis=1), b.max(axis=0))
    tol = 4 * (k + 4) * U_FMT[C] * S + slicing + 4 * U_FMT[C] * S
    d = orc.diff(got, ref)
    assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol)
    print(f"C={C} k={k}: err / sum|a||b| {float(np.max(np.abs(d) / S)):.3e}")
