"""The workload configurations at full size, checked through properties that hold at any
size (the oracle's own LU would take minutes to hours here):

  C1  DD n=64, unblocked (panel = n), 4M, x = 1: elementwise against the oracle
  C2  DD n=1024, panel 64, 3M and 4M, x = 1: eta, forward error against x = 1 and
      against the oracle's solution (kappa from the oracle's condition estimate),
      3M-vs-4M agreement and the imaginary-part residual growth of 3M
  C3  TD and QD n=2048, panel 64, A = U diag(sigma) V^H with sigma from 1 to 1e-30, four
      right-hand sides (ones, k + k i, two random DD columns): eta and forward error
      against kappa u; the same structure at n=96 elementwise against the oracle
  C4  DD n=4096, panel 128, rows scaled by 2^U(-20,20): 3M, INT8 split and the FP64
      split slice-count sweep, eta for each
  C5  DD n=2048, 16 right-hand sides, L = Re sum c^H x: the adjoint against the
      residual of A^H g_b = c, the rank-16 update, and quadruple-double central
      differences (step 2^-60) on 32 entries
  metric  DD / QD n=4096: eta of the 3M factorisation
  paper LU workload (Sec. 4) at n = 384-512: every update form against the oracle's
      solution and against x_k = k + k i

eta = ||b - A x||_inf / (||A||_inf ||x||_inf) always comes from an exact residual.
"""
import json
import os
import time
from fractions import Fraction

import numpy as np
import pytest

import synthgen
from helpers import U_FMT, to_dev, to_host

pytestmark = pytest.mark.gpu

# measured figures are printed, and also appended to configs.jsonl in the directory named
# by MPLU_TEST_RECORDS when that is set
OUT = os.environ.get("MPLU_TEST_RECORDS")


def record(name, **kw):
    if OUT:
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, "configs.jsonl"), "a") as f:
            f.write(json.dumps({"test": name, **kw}) + "\n")
    print(name, kw)


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


def gesv_gpu(mp, A, B, **kw):
    import torch

    T, Bd = to_dev(A), to_dev(B)
    sync()
    t0 = time.perf_counter()
    ipiv, info = mp.gesv(T, Bd, **kw)
    sync()
    dt = time.perf_counter() - t0
    return to_host(Bd), to_host(T), ipiv.cpu().numpy(), int(info.item()), dt


def fwd_err(X, Xt, orc):
    X, Xt = np.ascontiguousarray(X), np.ascontiguousarray(Xt)
    d = orc.diff(X, Xt)
    return float(np.abs(d).max() / np.abs(orc.hi_complex(Xt)).max())


def test_c1_unblocked_dd_n64(mp, orc):
    n, C = 64, 2
    A = orc.canon(synthgen.uniform(n, n, C, 0))
    xt = synthgen.ones(n, 1, C)
    b = orc.matmul_exact(A, xt)
    xo, LUo, ipo, _ = orc.gesv(A, b)
    x, LU, ip, info, _ = gesv_gpu(mp, A, b, panel=n, method="4m")
    assert info == 0 and np.array_equal(ip, ipo)
    kappa = orc.cond_inf_est(A, LUo, ipo)
    assert fwd_err(x, xo, orc) <= 10 * n * kappa * U_FMT[C]
    assert np.abs(orc.diff(LU, LUo)).max() <= 100 * n * U_FMT[C] * np.abs(orc.hi_complex(LUo)).max()
    eta = orc.backward_error(A, x, b)
    record("C1", eta=eta, fwd_vs_oracle=fwd_err(x, xo, orc))
    assert eta <= 10 * n * U_FMT[C]


def test_c2_dd_n1024_3m_vs_4m(mp, orc):
    n, C = 1024, 2
    A = orc.canon(synthgen.uniform(n, n, C, 0))
    xt = synthgen.ones(n, 1, C)
    b = orc.matmul_exact(A, xt)
    # the oracle's own solution and its condition estimate (Hager / Higham on A^H)
    xo, LUo, ipo, info_o = orc.gesv(A, b)
    assert info_o == 0
    kappa = orc.cond_inf_est(A, LUo, ipo)
    res = {}
    for method in ("3m", "4m"):
        gesv_gpu(mp, A, b, panel=64, method=method)  # warm-up
        x, _, _, info, dt = gesv_gpu(mp, A, b, panel=64, method=method)
        assert info == 0
        r = orc.resid(A, x, b)
        nA = np.abs(orc.hi_complex(A)).sum(axis=1).max()
        nx = np.abs(orc.hi_complex(x)).max()
        eta = float(np.abs(r).max() / (nA * nx))
        eta_im = float(np.abs(r.imag).max() / (nA * nx))
        fe = fwd_err(x, xt, orc)
        fo = fwd_err(x, xo, orc)
        res[method] = dict(eta=eta, eta_im=eta_im, fwd=fe, fwd_vs_oracle=fo, seconds=dt, x=x)
        assert eta <= 10 * n * U_FMT[C]
        assert fe <= 10 * n * kappa * U_FMT[C]
        assert fo <= 10 * n * kappa * U_FMT[C]
    agree = fwd_err(res["3m"]["x"], res["4m"]["x"], orc)
    assert agree <= 20 * n * kappa * U_FMT[C]
    record("C2", kappa=kappa, t3m_over_t4m=res["3m"]["seconds"] / res["4m"]["seconds"],
           **{f"{k}_{m}": v for m in res for k, v in res[m].items() if k != "x"},
           agree_3m_4m=agree)


@pytest.fixture(scope="module")
def c3_qd():
    import oracle

    n = 2048
    VL, VR = synthgen.householder_vectors(n, 32, 0)
    sig = synthgen.geometric_sigma(n, 4)
    return oracle.gen_illcond(n, 4, sig, VL, VR)


def c3_rhs(n, C, orc):
    X = np.zeros((2, C, 4, n))
    X[:, :, 0:1] = synthgen.ones(n, 1, C)
    X[:, :, 1:2] = synthgen.k_plus_ki(n, C)
    R = orc.canon(synthgen.uniform(n, 2, 2, 5))
    X[:, :2, 2:4] = R
    return X


@pytest.mark.parametrize("C", [3, 4])
def test_c3_illconditioned_n2048(mp, orc, c3_qd, C):
    n = 2048
    A = c3_qd if C == 4 else orc.round_to(c3_qd, 3)
    X = c3_rhs(n, C, orc)
    B = orc.matmul_exact(A, X)
    Xg, _, _, info, dt = gesv_gpu(mp, A, B, panel=64, method="3m")
    assert info == 0
    eta = orc.backward_error(A, Xg, B)
    kappa = n * 1e30            # kappa_inf <= n kappa_2, kappa_2 = 1e30 by construction
    fes = [fwd_err(Xg[:, :, k:k + 1], X[:, :, k:k + 1], orc) for k in range(4)]
    record("C3", C=C, eta=eta, fwd=fes, seconds=dt, bound_fwd=10 * n * kappa * U_FMT[C])
    assert eta <= 10 * n * U_FMT[C]
    assert max(fes) <= 10 * n * kappa * U_FMT[C]


@pytest.mark.parametrize("C", [3, 4])
def test_c3_structure_vs_oracle_n96(mp, orc, C):
    n = 96
    VL, VR = synthgen.householder_vectors(n, 32, 1)
    A = orc.gen_illcond(n, 4, synthgen.geometric_sigma(n, 4), VL, VR)
    if C == 3:
        A = orc.round_to(A, 3)
    X = c3_rhs(n, C, orc)
    B = orc.matmul_exact(A, X)
    Xo, LUo, ipo, _ = orc.gesv(A, B)
    Xg, LUg, ipg, info, _ = gesv_gpu(mp, A, B, panel=32, method="3m")
    assert info == 0
    kappa = n * 1e30
    assert fwd_err(Xg, Xo, orc) <= 10 * n * kappa * U_FMT[C]
    # factors of a matrix this ill-conditioned differ by up to kappa u, so check what
    # both must satisfy: P A = L U + E with |E| <= 10 n u |L||U| (exact product of L, U)
    for LU, ip in ((LUg, ipg), (LUo, ipo)):
        assert factor_backward_error(orc, A, LU, ip) <= 10 * n * U_FMT[C]
    assert orc.backward_error(A, Xg, B) <= 10 * n * U_FMT[C]


def factor_backward_error(orc, A, LU, ipiv):
    """max |P A - L U| / max (|L||U|), with L U formed exactly (rounded once)."""
    n, C = A.shape[2], A.shape[1]
    L = np.zeros_like(LU)
    U = np.zeros_like(LU)
    for j in range(n):
        L[:, :, j, j + 1:] = LU[:, :, j, j + 1:]
        U[:, :, j, :j + 1] = LU[:, :, j, :j + 1]
    L[0, 0, np.arange(n), np.arange(n)] = 1.0
    PA = A.copy()
    for k in range(n):
        p = ipiv[k] - 1
        if p != k:
            PA[:, :, :, [k, p]] = PA[:, :, :, [p, k]]
    R = orc.matmul_exact(L, U)
    d = orc.diff(np.ascontiguousarray(PA), R)
    LUmag = np.abs(orc.hi_complex(L)) @ np.abs(orc.hi_complex(U))
    return float(np.abs(d).max() / LUmag.max())


def test_c4_split_vs_3m_dd_n4096(mp, orc):
    n, C = 4096, 2
    A = orc.canon(synthgen.uniform(n, n, C, 0, row_exp=synthgen.row_exponents(n, 0)))
    b = orc.matmul_exact(A, synthgen.ones(n, 1, C))
    runs = [("3m", 0), ("split_i8", 0), ("split_f64", 6), ("split_f64", 5), ("split_f64", 4),
            ("split_f64", 3)]
    out = {}
    for method, S in runs:
        x, _, _, info, dt = gesv_gpu(mp, A, b, panel=128, method=method, n_slices=S)
        assert info == 0
        eta = orc.backward_error(A, x, b)
        out[f"{method}{'_S' + str(S) if S else ''}"] = dict(eta=eta, seconds=dt)
        if S in (0, 6):
            assert eta <= 10 * n * U_FMT[C], (method, S, eta)
    record("C4", **out)


def test_c5_adjoint_dd_n2048(mp, orc):
    import torch

    n, C, nrhs = 2048, 2, 16
    A = orc.canon(synthgen.uniform(n, n, C, 0))
    B = orc.canon(synthgen.uniform(n, nrhs, C, 1))
    c = orc.canon(synthgen.uniform(n, nrhs, C, 2))
    Ad = to_dev(A).requires_grad_(True)
    Bd = to_dev(B).requires_grad_(True)
    X = mp.solve(Ad, Bd)
    X.backward(to_dev(c))
    sync()
    gA, gB, Xh = to_host(Ad.grad), to_host(Bd.grad), to_host(X)
    # (1) g_b solves A^H g_b = c
    AH = np.ascontiguousarray(np.transpose(A, (0, 1, 3, 2)))
    AH[1] *= -1
    eta_adj = orc.backward_error(AH, gB, c)
    assert eta_adj <= 10 * n * U_FMT[C]
    # (2) g_A = -g_b x^H at sampled entries (exact rational check of the rank-16 update)
    ents = synthgen.sample_entries(n, 32, 3)

    def fz(P, i, j):
        return (sum(Fraction(float(v)) for v in P[0, :, j, i]),
                sum(Fraction(float(v)) for v in P[1, :, j, i]))

    for (i, j) in ents:
        er, ei, mag = Fraction(0), Fraction(0), 0.0
        for k in range(nrhs):
            gr, gi = fz(gB, i, k)
            xr, xi = fz(Xh, j, k)
            er -= gr * xr + gi * xi        # -(g conj(x))
            ei -= gi * xr - gr * xi
            mag += (abs(float(gr)) + abs(float(gi))) * (abs(float(xr)) + abs(float(xi)))
        got = fz(gA, i, j)
        assert abs(float(got[0] - er)) <= 64 * U_FMT[C] * mag
        assert abs(float(got[1] - ei)) <= 64 * U_FMT[C] * mag
    # (3) quadruple-double central differences, step 2^-60, on device-resident copies
    A4, B4, c4 = (np.zeros((2, 4) + P.shape[2:]) for P in (A, B, c))
    for P4, P in ((A4, A), (B4, B), (c4, c)):
        P4[:, :2] = P
    A4d, B4d, c4d = to_dev(A4), to_dev(B4), to_dev(c4)
    h = 2.0 ** -60

    def loss(part, i, j, sgn):
        T = A4d.clone()
        T[part, 2, j, i] = sgn * h      # A_ij +- h exactly (an extra component), renormalised
        mp.renorm_(T)
        Xd = B4d.clone()
        _, info = mp.gesv(T, Xd, panel=64, method="3m")
        G = to_host(mp.gemm(c4d, Xd, None, opA="C", method="4m"))
        assert int(info.item()) == 0
        return sum((sum(Fraction(float(v)) for v in G[0, :, k, k]) for k in range(nrhs)),
                   Fraction(0))

    worst = 0.0
    scale = Fraction(float(np.abs(orc.hi_complex(gA)).max()))
    for (i, j) in ents:
        for part in (0, 1):
            fd = (loss(part, i, j, 1.0) - loss(part, i, j, -1.0)) / (2 * Fraction(h))
            g = sum((Fraction(float(v)) for v in gA[part, :, j, i]), Fraction(0))
            worst = max(worst, float(abs(fd - g) / scale))   # compared exactly, then rounded
    record("C5", eta_adjoint=eta_adj, fd_rel_err=worst)
    assert worst <= 1e-20


@pytest.mark.parametrize("C", [2, 4])
def test_metric_eta_n4096(mp, orc, C):
    n = 4096
    A = orc.canon(synthgen.uniform(n, n, C, 0))
    b = orc.matmul_exact(A, synthgen.ones(n, 1, C))
    for panel in (64, 128):
        x, _, _, info, dt = gesv_gpu(mp, A, b, panel=panel, method="3m")
        assert info == 0
        eta = orc.backward_error(A, x, b)
        record("metric", C=C, panel=panel, eta=eta, seconds=dt)
        assert eta <= 10 * n * U_FMT[C]


@pytest.mark.parametrize("C", [2, 3, 4])
def test_matmul_paper_workload_n2048_sampled(mp, orc, C):
    """The matrix-product benchmark of Sec. 2.4 at the size the benchmark times (n = 2048,
    leading components uniform on [0, 1]) in every product form: a 24 x 24 block of
    sampled rows and columns of each GPU product against the oracle's product of the same
    rows and columns, elementwise within 4 (n + 4) u sum |a||b| (plus the slicing term of
    the split forms, 2^-(53C+2) below each row / column maximum; Strassen-Winograd within
    its normwise bound)."""
    import torch

    n = 2048
    A = orc.canon(synthgen.uniform(n, n, C, 11, lo=0.0, hi=1.0))
    B = orc.canon(synthgen.uniform(n, n, C, 12, lo=0.0, hi=1.0))
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(n, 24, replace=False))
    cols = np.sort(rng.choice(n, 24, replace=False))
    As = np.ascontiguousarray(A[:, :, :, rows])
    Bs = np.ascontiguousarray(B[:, :, cols, :])
    a = (np.abs(As[0, 0]) + np.abs(As[1, 0])).T
    b = (np.abs(Bs[0, 0]) + np.abs(Bs[1, 0])).T
    S = a @ b
    slicing = 16 * n * 2.0 ** (-53 * C - 2) * np.outer(
        (np.abs(A[0, 0]) + np.abs(A[1, 0])).T.max(axis=1)[rows],
        (np.abs(B[0, 0]) + np.abs(B[1, 0])).T.max(axis=0)[cols])
    amax = (np.abs(A[0, 0]) + np.abs(A[1, 0])).max()
    bmax = (np.abs(B[0, 0]) + np.abs(B[1, 0])).max()
    Ad, Bd = to_dev(A), to_dev(B)
    worst = {}
    for method in ("4m", "3m", "split_i8", "split_f64", "strassen"):
        ref = orc.gemm(As, Bs, None, method=4 if method == "4m" else 3, threads=0)
        got = to_host(mp.gemm(Ad, Bd, None, method=method))[:, :, cols][:, :, :, rows]
        d = orc.diff(np.ascontiguousarray(got), ref)
        tol = 4 * (n + 4) * U_FMT[C] * S + (slicing if method.startswith("split") else 0)
        if method == "strassen":   # normwise (one Winograd level): 64 (n + 4) u n max|a| max|b|
            tol = 64 * (n + 4) * U_FMT[C] * n * amax * bmax
        assert np.all(np.abs(d.real) <= tol) and np.all(np.abs(d.imag) <= tol), method
        worst[method] = float(np.max(np.abs(d) / S))
    record("matmul_n2048", C=C, err_over_sum_abs=worst)
    del Ad, Bd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("C,n", [(2, 512), (3, 384), (4, 384)])
def test_paper_lu_workload_vs_oracle(mp, orc, C, n):
    """The LU workload of Sec. 4 (leading components uniform on [0, 1], x_k = k + k i) at
    a size the oracle factors in seconds, with b = A x formed exactly and rounded once to
    the working format (the paper forms it at 2048 bits; exact-then-round is at least as
    good).  Every trailing-update form, panel 64: the solution elementwise against the
    oracle's solution and against x, each within 10 n kappa u (kappa from the oracle's
    condition estimate), eta within 10 n u by the exact residual, and the maximum relative
    error max_k |x_k - x*_k| / |x*_k| of the paper's tables recorded."""
    A = orc.canon(synthgen.uniform(n, n, C, 5, lo=0.0, hi=1.0))
    xt = synthgen.k_plus_ki(n, C)
    b = orc.matmul_exact(A, xt)
    xo, LUo, ipo, info_o = orc.gesv(A, b)
    assert info_o == 0
    kappa = orc.cond_inf_est(A, LUo, ipo)
    xmod = np.sqrt(2.0) * np.arange(1, n + 1)
    u = U_FMT[C]
    out = {}
    for method in ("4m", "3m", "split_i8", "split_f64"):
        x, _, _, info, _ = gesv_gpu(mp, A, b, panel=64, method=method)
        assert info == 0, method
        fo, fx = fwd_err(x, xo, orc), fwd_err(x, xt, orc)
        rel = float((np.abs(orc.diff(np.ascontiguousarray(x), xt))[:, 0] / xmod).max())
        eta = orc.backward_error(A, x, b)
        out[method] = dict(eta=eta, fwd_vs_oracle=fo, fwd=fx, max_rel_err=rel)
        assert fo <= 10 * n * kappa * u, method
        assert fx <= 10 * n * kappa * u, method
        assert eta <= 10 * n * u, method
    fo_oracle = fwd_err(xo, xt, orc)
    record("paper_lu", C=C, n=n, kappa=kappa, oracle_fwd=fo_oracle, **out)
