"""The C ABI: the library loads, exports every entry point declared in include/mplu.h,
and rejects bad arguments before touching the GPU (LAPACK-style -i codes)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "mplu.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(mplu_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def L():
    import paper_2403_16013_amd as m

    return m.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name


def test_version_and_strerror(L):
    assert L.mplu_version() >= 10000
    assert L.mplu_strerror(0) == b"success"
    assert L.mplu_strerror(-100) == b"workspace too small"
    assert L.mplu_strerror(-3) == b"invalid argument"


def test_argument_checks(L):
    import paper_2403_16013_amd as m

    z = m.ZMat(0x1000, 8, 64)
    null = m.ZMat(0, 8, 64)
    ip = ct.c_void_p(0x2000)
    inf = ct.c_void_p(0x3000)
    wk = ct.c_void_p(0x10000)
    # precision
    assert L.mplu_zgetrf(5, 8, 8, z, ip, inf, None, wk, 1 << 30, None) == -1
    assert L.mplu_zgetrf(2, -1, 8, z, ip, inf, None, wk, 1 << 30, None) == -2
    assert L.mplu_zgetrf(2, 8, -1, z, ip, inf, None, wk, 1 << 30, None) == -3
    assert L.mplu_zgetrf(2, 8, 8, null, ip, inf, None, wk, 1 << 30, None) == -4
    assert L.mplu_zgetrf(2, 9, 8, z, ip, inf, None, wk, 1 << 30, None) == -4   # ld < m
    assert L.mplu_zgetrf(2, 8, 9, z, ip, inf, None, wk, 1 << 30, None) == -4   # stride
    assert L.mplu_zgetrf(2, 8, 8, z, None, inf, None, wk, 1 << 30, None) == -5
    assert L.mplu_zgetrf(2, 8, 8, z, ip, None, None, wk, 1 << 30, None) == -6
    bad = m.Opts(-1, 1, 0, 0, 0)
    assert L.mplu_zgetrf(2, 8, 8, z, ip, inf, ct.byref(bad), wk, 1 << 30, None) == -7
    bad = m.Opts(64, 9, 0, 0, 0)
    assert L.mplu_zgetrf(2, 8, 8, z, ip, inf, ct.byref(bad), wk, 1 << 30, None) == -7
    # flags: only MPLU_FLAG_NO_LOOKAHEAD (1) and MPLU_FLAG_EXPIRE_WAITS (2) are defined
    for flags in (4, 1 | 8, 2 | 16, -1):
        bad = m.Opts(64, 1, 0, 0, flags)
        assert L.mplu_zgetrf(2, 8, 8, z, ip, inf, ct.byref(bad), wk, 1 << 30, None) == -7
        assert L.mplu_zgesv(2, 8, 1, z, ip, z, inf, ct.byref(bad), wk, 1 << 30, None) == -8
    assert m.FLAG_NO_LOOKAHEAD == 1 and m.FLAG_EXPIRE_WAITS == 2
    hdr = open(os.path.join(ROOT, "include", "mplu.h")).read()
    assert re.search(r"#define\s+MPLU_FLAG_NO_LOOKAHEAD\s+1\b", hdr)
    assert re.search(r"#define\s+MPLU_FLAG_EXPIRE_WAITS\s+2\b", hdr)
    # the options structure as the header declares it (the binding's copy must match)
    fields = re.search(r"typedef struct \{\s*int32_t panel;(.*?)\} mplu_opts_t;", hdr, re.S)
    names = re.findall(r"^\s*(?:int32_t|void \*)\s*(\w+);", "int32_t panel;" + fields.group(1),
                       re.M)
    assert names == [f[0] for f in m.Opts._fields_]
    assert ct.sizeof(m.Opts) == 32
    assert L.mplu_zgetrf(2, 8, 8, z, ip, inf, None, ct.c_void_p(0x10001), 1 << 30, None) == -8
    assert L.mplu_zgetrf(2, 8, 8, z, ip, inf, None, wk, 16, None) == -100
    assert L.mplu_zgetrs(2, b"X", 8, 1, z, ip, z, wk, 1 << 30, None) == -2
    assert L.mplu_zgetrs(2, b"N", 8, 1, z, None, z, wk, 1 << 30, None) == -6
    assert L.mplu_zgetrs(2, b"N", 8, 2, z, ip, m.ZMat(0x1000, 8, 8), wk, 1 << 30, None) == -7
    assert L.mplu_zgesv(2, 8, 1, z, ip, z, None, None, wk, 1 << 30, None) == -7
    assert L.mplu_zgemm(2, b"Q", b"N", 4, 4, 4, 1, z, z, 0, z, 0, None, wk, 0, None) == -2
    assert L.mplu_zgemm(2, b"N", b"N", 4, 4, 4, 2, z, z, 0, z, 0, None, wk, 0, None) == -7
    assert L.mplu_zgemm(2, b"N", b"N", 4, 4, 4, 1, z, z, 2, z, 0, None, wk, 0, None) == -10
    assert L.mplu_zgemm(2, b"N", b"N", 4, 4, 4, 1, z, z, 0, z, 7, None, wk, 0, None) == -12
    # real matrices
    d = m.DMat(0x1000, 8, 64)
    dnull = m.DMat(0, 8, 64)
    assert L.mplu_dgetrf(5, 8, 8, d, ip, inf, None, wk, 1 << 30, None) == -1
    assert L.mplu_dgetrf(2, 9, 8, d, ip, inf, None, wk, 1 << 30, None) == -4
    assert L.mplu_dgetrf(2, 8, 8, dnull, ip, inf, None, wk, 1 << 30, None) == -4
    assert L.mplu_dgetrf(2, 8, 8, d, None, inf, None, wk, 1 << 30, None) == -5
    assert L.mplu_dgetrf(2, 8, 8, d, ip, None, None, wk, 1 << 30, None) == -6
    bad = m.Opts(-1, 1, 0, 0, 0)
    assert L.mplu_dgetrf(2, 8, 8, d, ip, inf, ct.byref(bad), wk, 1 << 30, None) == -7
    assert L.mplu_dgesv(2, 8, 1, d, ip, d, inf, ct.byref(bad), wk, 1 << 30, None) == -8
    split = m.Opts(64, 3, 99, 0, 0)   # a slice count the split kernels do not have
    assert L.mplu_dgetrf(2, 8, 8, d, ip, inf, ct.byref(split), wk, 1 << 30, None) == -102
    assert L.mplu_dgesv(2, 8, 1, d, ip, d, inf, ct.byref(split), wk, 1 << 30, None) == -102
    assert L.mplu_zgetrf(2, 8, 8, z, ip, inf, ct.byref(split), wk, 1 << 30, None) == -102
    assert L.mplu_dgetrf(2, 8, 8, d, ip, inf, None, ct.c_void_p(0x10001), 1 << 30, None) == -8
    assert L.mplu_dgetrf(2, 8, 8, d, ip, inf, None, wk, 16, None) == -100
    assert L.mplu_dgetrs(2, b"C", 8, 1, d, ip, d, wk, 1 << 30, None) == -2
    assert L.mplu_dgetrs(2, b"N", 8, 1, d, None, d, wk, 1 << 30, None) == -6
    assert L.mplu_dgetrs(2, b"N", 8, 1, d, ip, d, wk, 16, None) == -100
    assert L.mplu_dgesv(2, 8, 1, d, ip, d, None, None, wk, 1 << 30, None) == -7
    assert L.mplu_dgemm(2, b"C", b"N", 4, 4, 4, 1, d, d, 0, d, None) == -2
    assert L.mplu_dgemm(2, b"N", b"N", 4, 4, 4, 2, d, d, 0, d, None) == -7
    assert L.mplu_dgemm(2, b"N", b"N", 4, 4, 4, 1, d, d, 2, d, None) == -10
    assert L.mplu_dgemm(2, b"N", b"N", 4, 4, 4, 1, d, d, 0, dnull, None) == -11
    # Strassen-Winograd: 'N', 'N' products; a trailing-update choice of the complex LU
    # only (its workspace holds the update's product and two half-size operand sums)
    assert L.mplu_zgemm(2, b"T", b"N", 4, 4, 4, 1, z, z, 0, z, 4, None, wk, 1 << 30, None) == -102
    assert L.mplu_zgemm(2, b"N", b"N", 4, 4, 4, 1, z, z, 0, z, 4, None, wk, 16, None) == -100
    assert L.mplu_zgemm(2, b"N", b"N", 4, 4, 4, 1, z, z, 0, z, 5, None, wk, 0, None) == -12
    st = m.Opts(64, 4, 0, 0, 0)
    assert L.mplu_dgetrf(2, 8, 8, d, ip, inf, ct.byref(st), wk, 1 << 30, None) == -102
    assert L.mplu_dgesv(2, 8, 1, d, ip, d, inf, ct.byref(st), wk, 1 << 30, None) == -102
    assert L.mplu_zgetrf(2, 8, 8, z, ip, inf, ct.byref(st), wk, 16, None) == -100
    three = m.Opts(64, 1, 0, 0, 0)
    ws3, wss = ct.c_size_t(), ct.c_size_t()
    assert L.mplu_zgetrf_wsbytes(2, 4096, 4096, ct.byref(three), ct.byref(ws3)) == 0
    assert L.mplu_zgetrf_wsbytes(2, 4096, 4096, ct.byref(st), ct.byref(wss)) == 0
    assert wss.value - ws3.value >= 2 * 2 * 8 * 4096 * 4096  # the m x n product W
    # panel widths above 128 (the LDS-resident panel) are refused, not clamped; a width
    # >= min(m, n) asks for the unblocked LU, possible only for min(m, n) <= 128
    big = m.ZMat(0x1000, 4096, 4096 * 4096)
    for pw, nn in ((256, 512), (129, 4096), (4096, 4096), (200, 200)):
        wide = m.Opts(pw, 1, 0, 0, 0)
        assert L.mplu_zgetrf(2, nn, nn, big, ip, inf, ct.byref(wide), wk, 1 << 40, None) == -102
    # the no-allocation gesv: the same argument checks, and the static scratch limit,
    # all decided before anything touches the GPU
    assert L.mplu_zgesv_noalloc(5, 8, 1, z, ip, z, inf, None, None) == -1
    assert L.mplu_zgesv_noalloc(2, -1, 1, z, ip, z, inf, None, None) == -2
    assert L.mplu_zgesv_noalloc(2, 8, -1, z, ip, z, inf, None, None) == -3
    assert L.mplu_zgesv_noalloc(2, 8, 1, null, ip, z, inf, None, None) == -4
    assert L.mplu_zgesv_noalloc(2, 8, 1, z, None, z, inf, None, None) == -5
    assert L.mplu_zgesv_noalloc(2, 8, 2, z, ip, m.ZMat(0x1000, 8, 8), inf, None, None) == -6
    assert L.mplu_zgesv_noalloc(2, 8, 1, z, ip, z, None, None, None) == -7
    assert L.mplu_zgesv_noalloc(2, 8, 1, z, ip, z, inf, ct.byref(bad), None) == -8
    scratch = 16 << 20
    sz = ct.c_size_t()
    for C, n, nrhs, opt in ((4, 4096, 64, None), (2, 4096, 1, m.Opts(64, 3, 0, 0, 0)),
                            (2, 8192, 200, None)):
        assert L.mplu_zgesv_wsbytes(C, n, nrhs, ct.byref(opt) if opt else None,
                                    ct.byref(sz)) == 0
        assert sz.value > scratch
        A = m.ZMat(0x1000, n, n * n)
        Bm = m.ZMat(0x1000, n, n * nrhs)
        rc = L.mplu_zgesv_noalloc(C, n, nrhs, A, ip, Bm, inf,
                                  ct.byref(opt) if opt else None, None)
        assert rc == -103, (C, n, nrhs, rc)
    assert L.mplu_strerror(-103).startswith(b"workspace need exceeds the static scratch")
    assert L.mplu_zrenorm(2, 8, 8, null, None) == -4
    assert L.mplu_zconvert(2, 7, 8, 8, z, z, None) == -2


def test_workspace_queries(L):
    import paper_2403_16013_amd as m

    sz = ct.c_size_t()
    assert L.mplu_zgetrf_wsbytes(2, 4096, 4096, None, ct.byref(sz)) == 0
    a = sz.value
    o = m.Opts(128, 1, 0, 0, 0)
    assert L.mplu_zgetrf_wsbytes(4, 4096, 4096, ct.byref(o), ct.byref(sz)) == 0
    assert sz.value > a > 0
    # the split methods add slice workspaces for the rest and for the next panel's columns
    o3 = m.Opts(128, 3, 0, 0, 0)
    assert L.mplu_zgetrf_wsbytes(2, 4096, 4096, ct.byref(o3), ct.byref(sz)) == 0
    i8 = sz.value
    assert i8 > a
    g = ct.c_size_t()
    assert L.mplu_zgemm_wsbytes(2, 4096, 4096, 128, 3, ct.byref(o3), ct.byref(g)) == 0
    assert i8 >= g.value
    # INT8 split products deeper than the INT32 limit of a combined level sum (5 248 for
    # QD: three times 64 S 65^2 per 64-deep chunk below 2^31) run in pieces of that depth,
    # so their workspace stops growing there
    deep, piece = ct.c_size_t(), ct.c_size_t()
    assert L.mplu_zgemm_wsbytes(4, 64, 64, 40000, 3, None, ct.byref(deep)) == 0
    assert L.mplu_zgemm_wsbytes(4, 64, 64, 5248, 3, None, ct.byref(piece)) == 0
    assert deep.value == piece.value
    assert L.mplu_zgemm_wsbytes(4, 64, 64, 5312, 3, None, ct.byref(deep)) == 0
    assert L.mplu_zgemm_wsbytes(4, 64, 64, 5184, 3, None, ct.byref(g)) == 0
    assert g.value < piece.value
    assert L.mplu_zgetrs_wsbytes(2, 100, 3, ct.byref(sz)) == 0
    assert sz.value >= 100 * 3 * 4 * 8
    assert L.mplu_zgesv_wsbytes(3, 100, 3, None, ct.byref(sz)) == 0
    # Strassen-Winograd: the m x n product and two half-size operand sums
    assert L.mplu_zgemm_wsbytes(3, 100, 80, 60, 4, None, ct.byref(g)) == 0
    assert g.value >= 2 * 3 * 8 * (100 * 80 + 50 * 30 + 30 * 40)
    # real: the same workspaces as the complex routines (which bound the real kernels')
    zf, df = ct.c_size_t(), ct.c_size_t()
    assert L.mplu_zgetrf_wsbytes(2, 300, 200, None, ct.byref(zf)) == 0
    assert L.mplu_dgetrf_wsbytes(2, 300, 200, None, ct.byref(df)) == 0
    assert df.value == zf.value > 0
    assert L.mplu_zgetrs_wsbytes(4, 100, 3, ct.byref(zf)) == 0
    assert L.mplu_dgetrs_wsbytes(4, 100, 3, ct.byref(df)) == 0
    assert df.value == zf.value >= 100 * 3 * 4 * 8
    assert L.mplu_dgesv_wsbytes(3, 100, 3, None, ct.byref(df)) == 0
    assert df.value == sz.value
