"""CPU oracle for complex multi-component LU (test infrastructure only).

The oracle is a plain, slow, exact-then-round implementation written from the paper
(Kouya, "Performance evaluation of accelerated complex multiple-precision LU
decomposition"): the unblocked "Normal LU" of Sec. 3 with partial pivoting and 4M complex
arithmetic (Eq. 4m), forward/backward substitution, and the 3M / 4M complex matrix
products of Sec. 2.1 (Eq. 3m_cemm / Eq. 4m).  Every operation rounds the exact result
greedily to C binary64 components (see ``mpo.c``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The GPU library never does, and shares no code with it.

Arrays use the plane layout of the library: float64 numpy arrays of shape
``(2, C, ncols, ld)``; plane ``(ri, c)`` holds component ``c`` of the real (ri=0) or
imaginary (ri=1) part, and element (i, j) sits at ``[ri, c, j, i]`` (column-major).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "mpo.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile mpo.c into liboracle.so (gcc, OpenMP, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fno-strict-aliasing", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = ct.CDLL(_LIB_PATH)
        d = ct.POINTER(ct.c_double)
        i32p = ct.POINTER(ct.c_int32)
        i64 = ct.c_int64
        for name in ("orc_mp_add", "orc_mp_sub", "orc_mp_mul", "orc_mp_div"):
            getattr(_lib, name).argtypes = [ct.c_int, d, d, d]
            getattr(_lib, name).restype = None
        _lib.orc_mp_round.argtypes = [ct.c_int, ct.c_int, d, d]
        _lib.orc_mp_round.restype = None
        _lib.orc_z_mul4m.argtypes = [ct.c_int, d, d, d]
        _lib.orc_z_mul4m.restype = None
        _lib.orc_z_recip.argtypes = [ct.c_int, d, d]
        _lib.orc_z_recip.restype = None
        _lib.orc_z_cabs1_cmp.argtypes = [ct.c_int, d, d]
        _lib.orc_z_cabs1_cmp.restype = ct.c_int
        _lib.orc_threads.argtypes = [ct.c_int]
        _lib.orc_threads.restype = ct.c_int
        _lib.orc_zcanon.argtypes = [ct.c_int, i64, i64, d, i64, i64]
        _lib.orc_zround.argtypes = [ct.c_int, ct.c_int, i64, i64, d, i64, i64, d, i64, i64]
        _lib.orc_zdiff.argtypes = [ct.c_int, ct.c_int, i64, i64, d, i64, i64, d, i64, i64, d, d]
        _lib.orc_zgetf2.argtypes = [ct.c_int, i64, i64, d, i64, i64, i32p, i32p, i64, ct.c_int]
        _lib.orc_zgetrs.argtypes = [ct.c_int, ct.c_char, i64, i64, d, i64, i64, i32p, d, i64,
                                    i64, ct.c_int]
        _lib.orc_zgemm.argtypes = [ct.c_int, ct.c_int, ct.c_char, ct.c_char, i64, i64, i64,
                                   ct.c_int, d, i64, i64, d, i64, i64, ct.c_int, d, i64, i64,
                                   ct.c_int]
        _lib.orc_zmatmul_exact.argtypes = [ct.c_int, i64, i64, i64, d, i64, i64, d, i64, i64,
                                           d, i64, i64, ct.c_int]
        _lib.orc_zresid.argtypes = [ct.c_int, ct.c_int, ct.c_int, i64, i64, d, i64, i64, d,
                                    i64, i64, d, i64, i64, d, d, ct.c_int]
        _lib.orc_gen_illcond.argtypes = [ct.c_int, i64, d, ct.c_int, d, d, d, i64, i64,
                                         ct.c_int]
        for name in ("orc_zcanon", "orc_zround", "orc_zdiff", "orc_zgetf2", "orc_zgetrs",
                     "orc_zgemm", "orc_zmatmul_exact", "orc_zresid", "orc_gen_illcond"):
            getattr(_lib, name).restype = ct.c_int
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_int32))


def _geom(P: np.ndarray):
    """(C, ncols, ld, plane_stride) of a plane array."""
    assert P.ndim == 4 and P.shape[0] == 2 and P.flags.c_contiguous and P.dtype == np.float64
    C, ncols, ld = P.shape[1], P.shape[2], P.shape[3]
    return C, ncols, ld, ncols * ld


def set_threads(n: int = 0) -> int:
    """Set OpenMP threads (0 keeps the current setting); returns the active count."""
    return _load().orc_threads(int(n))


# ---------------------------------------------------------------- scalar operations
def _vec(a, C):
    v = np.zeros(4, dtype=np.float64)
    v[: len(a)] = a
    return v


def mp_add(a, b, C):
    o = np.zeros(4)
    _load().orc_mp_add(C, _dp(_vec(a, C)), _dp(_vec(b, C)), _dp(o))
    return o[:C].copy()


def mp_sub(a, b, C):
    o = np.zeros(4)
    _load().orc_mp_sub(C, _dp(_vec(a, C)), _dp(_vec(b, C)), _dp(o))
    return o[:C].copy()


def mp_mul(a, b, C):
    o = np.zeros(4)
    _load().orc_mp_mul(C, _dp(_vec(a, C)), _dp(_vec(b, C)), _dp(o))
    return o[:C].copy()


def mp_div(a, b, C):
    o = np.zeros(4)
    _load().orc_mp_div(C, _dp(_vec(a, C)), _dp(_vec(b, C)), _dp(o))
    return o[:C].copy()


def mp_round(values, C):
    v = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
    o = np.zeros(4)
    _load().orc_mp_round(C, len(v), _dp(v), _dp(o))
    return o[:C].copy()


def _zvec(z, C):
    v = np.zeros(8)
    v[:C] = z[0]
    v[C:2 * C] = z[1]
    return v


def z_mul4m(a, b, C):
    """a, b: (re_components, im_components); returns the same form."""
    o = np.zeros(8)
    _load().orc_z_mul4m(C, _dp(_zvec(a, C)), _dp(_zvec(b, C)), _dp(o))
    return o[:C].copy(), o[C:2 * C].copy()


def z_recip(a, C):
    o = np.zeros(8)
    _load().orc_z_recip(C, _dp(_zvec(a, C)), _dp(o))
    return o[:C].copy(), o[C:2 * C].copy()


def z_cabs1_cmp(a, b, C):
    return _load().orc_z_cabs1_cmp(C, _dp(_zvec(a, C)), _dp(_zvec(b, C)))


# ---------------------------------------------------------------- matrix operations
def canon(P: np.ndarray, m: int | None = None) -> np.ndarray:
    """Canonicalise every element (greedy RN of its exact value); returns a new array."""
    P = np.ascontiguousarray(P, dtype=np.float64).copy()
    C, ncols, ld, ps = _geom(P)
    m = ld if m is None else m
    _load().orc_zcanon(C, m, ncols, _dp(P), ld, ps)
    return P


def round_to(P: np.ndarray, Cout: int, m: int | None = None) -> np.ndarray:
    C, ncols, ld, ps = _geom(P)
    m = ld if m is None else m
    out = np.zeros((2, Cout, ncols, ld))
    _load().orc_zround(C, Cout, m, ncols, _dp(P), ld, ps, _dp(out), ld, ncols * ld)
    return out


def diff(X: np.ndarray, Y: np.ndarray, m: int | None = None) -> np.ndarray:
    """Complex array RN(X - Y) computed exactly, shape (m, ncols)."""
    CX, ncols, ldx, psx = _geom(X)
    CY, ncols2, ldy, psy = _geom(Y)
    assert ncols == ncols2
    m = min(ldx, ldy) if m is None else m
    re = np.zeros((ncols, m))
    im = np.zeros((ncols, m))
    _load().orc_zdiff(CX, CY, m, ncols, _dp(X), ldx, psx, _dp(Y), ldy, psy, _dp(re), _dp(im))
    return (re + 1j * im).T.copy()


def getf2(P: np.ndarray, m: int | None = None, kmax: int = -1, threads: int = 0):
    """Unblocked LU with partial pivoting (Sec. 3 "Normal LU", LAPACK getf2 semantics).

    Returns (LU, ipiv (1-based int32), info)."""
    LU = np.ascontiguousarray(P, dtype=np.float64).copy()
    C, n, ld, ps = _geom(LU)
    m = ld if m is None else m
    ipiv = np.zeros(max(1, min(m, n)), dtype=np.int32)
    info = np.zeros(1, dtype=np.int32)
    rc = _load().orc_zgetf2(C, m, n, _dp(LU), ld, ps, _ip(ipiv), _ip(info), kmax, threads)
    if rc != 0:
        raise RuntimeError(f"orc_zgetf2 failed: {rc}")
    return LU, ipiv[: min(m, n)], int(info[0])


def getrs(LU: np.ndarray, ipiv: np.ndarray, B: np.ndarray, trans: str = "N",
          threads: int = 0) -> np.ndarray:
    """Solve A X = B ('N') or A^H X = B ('C') with getf2's factors; returns X."""
    C, n, ld, ps = _geom(LU)
    X = np.ascontiguousarray(B, dtype=np.float64).copy()
    CB, nrhs, ldb, psb = _geom(X)
    assert CB == C
    ipv = np.ascontiguousarray(ipiv, dtype=np.int32)
    rc = _load().orc_zgetrs(C, trans.encode(), n, nrhs, _dp(LU), ld, ps, _ip(ipv), _dp(X), ldb,
                            psb, threads)
    if rc != 0:
        raise RuntimeError(f"orc_zgetrs failed: {rc}")
    return X


def gesv(A: np.ndarray, B: np.ndarray, threads: int = 0):
    LU, ipiv, info = getf2(A, threads=threads)
    return getrs(LU, ipiv, B, "N", threads=threads), LU, ipiv, info


def gemm(A: np.ndarray, B: np.ndarray, Cm: np.ndarray | None, method: int = 4, opA: str = "N",
         opB: str = "N", alpha_sign: int = 1, m: int | None = None, n: int | None = None,
         k: int | None = None, threads: int = 0) -> np.ndarray:
    """Cm := beta*Cm + alpha*op(A)*op(B), beta = 1 if Cm is given else 0 (Eq. 3m_cemm / 4m)."""
    CA, acols, lda, psa = _geom(A)
    CB_, bcols, ldb, psb = _geom(B)
    assert CA == CB_
    C = CA
    if m is None:
        m = lda if opA == "N" else acols
    if k is None:
        k = acols if opA == "N" else lda
    if n is None:
        n = bcols if opB == "N" else ldb
    beta = 1
    if Cm is None:
        beta = 0
        Cm = np.zeros((2, C, n, m))
    out = np.ascontiguousarray(Cm, dtype=np.float64).copy()
    _, ccols, ldc, psc = _geom(out)
    rc = _load().orc_zgemm(C, method, opA.encode(), opB.encode(), m, n, k, alpha_sign, _dp(A),
                           lda, psa, _dp(B), ldb, psb, beta, _dp(out), ldc, psc, threads)
    if rc != 0:
        raise RuntimeError(f"orc_zgemm failed: {rc}")
    return out


def matmul_exact(A: np.ndarray, X: np.ndarray, Cout: int | None = None, threads: int = 0):
    """B = RN(A X) with each part of each element rounded once from the exact value."""
    C, n, lda, psa = _geom(A)
    CX, nrhs, ldx, psx = _geom(X)
    assert CX == C
    m = lda
    B = np.zeros((2, C, nrhs, m))
    _load().orc_zmatmul_exact(C, m, n, nrhs, _dp(A), lda, psa, _dp(X), ldx, psx, _dp(B), m,
                              nrhs * m, threads)
    if Cout is not None and Cout != C:
        B = round_to(B, Cout)
    return B


def resid(A: np.ndarray, X: np.ndarray, B: np.ndarray, threads: int = 0) -> np.ndarray:
    """Exact residual b - A x rounded to complex128, shape (n, nrhs)."""
    CA, n, lda, psa = _geom(A)
    CX, nrhs, ldx, psx = _geom(X)
    CB, nrhs2, ldb, psb = _geom(B)
    assert nrhs == nrhs2
    re = np.zeros((nrhs, n))
    im = np.zeros((nrhs, n))
    _load().orc_zresid(CA, CX, CB, n, nrhs, _dp(A), lda, psa, _dp(X), ldx, psx, _dp(B), ldb,
                       psb, _dp(re), _dp(im), threads)
    return (re + 1j * im).T.copy()


def backward_error(A: np.ndarray, X: np.ndarray, B: np.ndarray, threads: int = 0) -> float:
    """eta = ||b - A x||_inf / (||A||_inf ||x||_inf), exact residual, complex modulus."""
    r = resid(A, X, B, threads=threads)
    Ah = hi_complex(A)
    Xh = hi_complex(X)
    nA = np.abs(Ah).sum(axis=1).max()
    nx = np.abs(Xh).max()
    nr = np.abs(r).max()
    return float(nr / (nA * nx)) if nA > 0 and nx > 0 else float(nr)


def hi_complex(P: np.ndarray) -> np.ndarray:
    """Leading components as a complex128 (rows x cols) matrix."""
    return (P[0, 0] + 1j * P[1, 0]).T.copy()


def gen_illcond(n: int, C: int, sigma: np.ndarray, VL: np.ndarray, VR: np.ndarray,
                threads: int = 0) -> np.ndarray:
    """A = U diag(sigma) V^H with U, V products of Householder reflectors (see mpo.c).

    sigma: (n, C) real components; VL, VR: complex (nrefl, n) exact doubles."""
    nrefl = VL.shape[0]
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    assert s.shape == (n, C)

    def pack(V):
        out = np.zeros((nrefl, 2, n))
        out[:, 0] = V.real
        out[:, 1] = V.imag
        return out

    vl, vr = pack(VL), pack(VR)
    A = np.zeros((2, C, n, n))
    rc = _load().orc_gen_illcond(C, n, _dp(s), nrefl, _dp(vl), _dp(vr), _dp(A), n, n * n,
                                 threads)
    if rc != 0:
        raise RuntimeError(f"orc_gen_illcond failed: {rc}")
    return A


def solve_grad(LU: np.ndarray, ipiv: np.ndarray, X: np.ndarray, Gx: np.ndarray,
               threads: int = 0):
    """Gradient of a real loss through x = A^-1 b, from the oracle's own factors.

    With the complex convention g = dL/dRe + i dL/dIm, differentiating A x = b gives
        g_b = A^-H g_x                 (a conjugate-transpose solve with getf2's factors)
        g_A = -g_b x^H                 (each element the exact product, rounded once)
    LU, ipiv: getf2's output for A; X: the solution (n x nrhs); Gx: dL/dx (n x nrhs).
    Returns (g_b, g_A) as plane arrays of the format of LU."""
    C, n, ld, _ = _geom(LU)
    _, nrhs, _, _ = _geom(Gx)
    Gb = getrs(LU, ipiv, Gx, "C", threads=threads)
    GA = gemm(Gb, X, None, method=4, opA="N", opB="C", alpha_sign=-1, m=n, n=n, k=nrhs,
              threads=threads)
    return Gb, GA


def _planes_of(z: np.ndarray, C: int) -> np.ndarray:
    """complex128 vector -> (2, C, 1, n) planes with zero lower components."""
    P = np.zeros((2, C, 1, z.shape[0]))
    P[0, 0, 0] = z.real
    P[1, 0, 0] = z.imag
    return P


def inv_norm1_est(LU: np.ndarray, ipiv: np.ndarray, trans: str = "N", itmax: int = 5,
                  threads: int = 0) -> float:
    """Estimate ||B||_1 for B = A^-1 (trans 'N') or B = A^-H (trans 'C') from getf2's
    factors, by the 1-norm power method of Hager (1984) with Higham's (1988) refinements
    for complex matrices: it only needs products with B and B^H, i.e. solves with A.

      x = e / n;  repeat:  y = B x,  xi_i = y_i / |y_i| (1 where y_i = 0),  z = B^H xi;
                           stop when ||z||_inf <= Re(z^H x) or the index repeats;
                           otherwise x = e_j with j the first index maximising |z_j|;
      then compare with 2 ||B w||_1 / (3 n) for w_i = (-1)^i (1 + i / (n - 1)), which
      guards against the cases where the power method stalls.

    The solves run in the oracle's multi-component arithmetic; the norms of the leading
    components suffice for an estimate.  The value is a lower bound of ||B||_1 (up to
    rounding), usually equal to it."""
    C, n, _, _ = _geom(LU)
    if n == 0:
        return 0.0
    other = "C" if trans == "N" else "N"

    def apply(z, tr):
        out = getrs(LU, ipiv, _planes_of(z, C), tr, threads=threads)
        return out[0, 0, 0] + 1j * out[1, 0, 0]

    x = np.full(n, 1.0 / n, dtype=complex)
    est, jlast = 0.0, -1
    for it in range(itmax):
        y = apply(x, trans)
        new = float(np.abs(y).sum())
        if it > 0 and new <= est:
            break
        est = new
        a = np.abs(y)
        xi = np.where(a > 0, y / np.where(a > 0, a, 1.0), 1.0)
        z = apply(xi, other)
        j = int(np.argmax(np.abs(z)))
        if np.abs(z).max() <= float(np.real(np.vdot(z, x))) or j == jlast:
            break
        x = np.zeros(n, dtype=complex)
        x[j] = 1.0
        jlast = j
    i = np.arange(n, dtype=float)
    w = ((-1.0) ** i) * (1.0 + i / max(1, n - 1))
    alt = 2.0 * float(np.abs(apply(w.astype(complex), trans)).sum()) / (3.0 * n)
    return max(est, alt)


def cond_inf_est(A: np.ndarray, LU: np.ndarray, ipiv: np.ndarray, threads: int = 0) -> float:
    """kappa_inf(A) = ||A||_inf ||A^-1||_inf, the second factor estimated as ||A^-H||_1
    (inv_norm1_est on A^H) from getf2's factors of A; ||A||_inf from the leading
    components (complex modulus)."""
    nA = float(np.abs(hi_complex(A)).sum(axis=1).max())
    return nA * inv_norm1_est(LU, ipiv, "C", threads=threads)
