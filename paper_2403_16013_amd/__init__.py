"""Complex multi-component (DD / TD / QD) LU with partial pivoting on MI355X.

Thin ctypes binding over ``libmplu.so`` (declared in ``include/mplu.h``).  Every step of
the factorisation and the solves runs in the library's HIP kernels; this module only
marshals torch tensors (device memory) and the current HIP stream.  It never computes.

Matrices are float64 CUDA tensors of shape ``(2, C, ncols, ld)``: plane ``[ri, c]`` is
component ``c`` of the real (ri = 0) or imaginary (ri = 1) part, column-major, so element
(i, j) is ``T[ri, c, j, i]``.  ``C`` = 2 (double-double), 3 (triple-double) or
4 (quadruple-double).
"""
from __future__ import annotations

import ctypes as ct
import os

import torch

__all__ = ["lib", "renorm_", "convert", "getrf", "getrs", "gesv", "gesv_noalloc", "gemm",
           "solve",
           "lu_factor", "lu_solve",
           "dgetrf", "dgetrs", "dgesv", "dgemm",
           "GEMM_4M", "GEMM_3M", "GEMM_SPLIT_F64", "GEMM_SPLIT_I8", "GEMM_STRASSEN",
           "MPLUError"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmplu.so")

GEMM_4M, GEMM_3M, GEMM_SPLIT_F64, GEMM_SPLIT_I8, GEMM_STRASSEN = 0, 1, 2, 3, 4
_METHODS = {"4m": GEMM_4M, "3m": GEMM_3M, "split_f64": GEMM_SPLIT_F64,
            "split_i8": GEMM_SPLIT_I8, "strassen": GEMM_STRASSEN}


class MPLUError(RuntimeError):
    pass


class ZMat(ct.Structure):
    _fields_ = [("planes", ct.c_void_p), ("ld", ct.c_int64), ("plane_stride", ct.c_int64)]


class DMat(ct.Structure):
    _fields_ = [("planes", ct.c_void_p), ("ld", ct.c_int64), ("plane_stride", ct.c_int64)]


class Opts(ct.Structure):
    _fields_ = [("panel", ct.c_int32), ("gemm", ct.c_int32), ("n_slices", ct.c_int32),
                ("slice_bits", ct.c_int32), ("flags", ct.c_int32), ("aux_stream", ct.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise MPLUError(f"{_LIB_PATH} is missing: build it with "
                        "`python -m paper_2403_16013_amd._build`")
    L = ct.CDLL(_LIB_PATH)
    i64, vp, sz = ct.c_int64, ct.c_void_p, ct.c_size_t
    i32p = ct.c_void_p
    L.mplu_version.restype = ct.c_int
    L.mplu_strerror.argtypes = [ct.c_int]
    L.mplu_strerror.restype = ct.c_char_p
    L.mplu_zrenorm.argtypes = [ct.c_int, i64, i64, ZMat, vp]
    L.mplu_zconvert.argtypes = [ct.c_int, ct.c_int, i64, i64, ZMat, ZMat, vp]
    L.mplu_zgetrf_wsbytes.argtypes = [ct.c_int, i64, i64, ct.POINTER(Opts), ct.POINTER(sz)]
    L.mplu_zgetrf.argtypes = [ct.c_int, i64, i64, ZMat, i32p, i32p, ct.POINTER(Opts), vp, sz, vp]
    L.mplu_zgetrs_wsbytes.argtypes = [ct.c_int, i64, i64, ct.POINTER(sz)]
    L.mplu_zgetrs.argtypes = [ct.c_int, ct.c_char, i64, i64, ZMat, i32p, ZMat, vp, sz, vp]
    L.mplu_zgesv_wsbytes.argtypes = [ct.c_int, i64, i64, ct.POINTER(Opts), ct.POINTER(sz)]
    L.mplu_zgesv.argtypes = [ct.c_int, i64, i64, ZMat, i32p, ZMat, i32p, ct.POINTER(Opts), vp,
                             sz, vp]
    L.mplu_zgesv_noalloc.argtypes = [ct.c_int, i64, i64, ZMat, i32p, ZMat, i32p,
                                     ct.POINTER(Opts), vp]
    L.mplu_zgemm_wsbytes.argtypes = [ct.c_int, i64, i64, i64, ct.c_int, ct.POINTER(Opts),
                                     ct.POINTER(sz)]
    L.mplu_zgemm.argtypes = [ct.c_int, ct.c_char, ct.c_char, i64, i64, i64, ct.c_int, ZMat,
                             ZMat, ct.c_int, ZMat, ct.c_int, ct.POINTER(Opts), vp, sz, vp]
    L.mplu_dgetrf_wsbytes.argtypes = [ct.c_int, i64, i64, ct.POINTER(Opts), ct.POINTER(sz)]
    L.mplu_dgetrf.argtypes = [ct.c_int, i64, i64, DMat, i32p, i32p, ct.POINTER(Opts), vp, sz, vp]
    L.mplu_dgetrs_wsbytes.argtypes = [ct.c_int, i64, i64, ct.POINTER(sz)]
    L.mplu_dgetrs.argtypes = [ct.c_int, ct.c_char, i64, i64, DMat, i32p, DMat, vp, sz, vp]
    L.mplu_dgesv_wsbytes.argtypes = [ct.c_int, i64, i64, ct.POINTER(Opts), ct.POINTER(sz)]
    L.mplu_dgesv.argtypes = [ct.c_int, i64, i64, DMat, i32p, DMat, i32p, ct.POINTER(Opts), vp,
                             sz, vp]
    L.mplu_dgemm.argtypes = [ct.c_int, ct.c_char, ct.c_char, i64, i64, i64, ct.c_int, DMat,
                             DMat, ct.c_int, DMat, vp]
    for name in ("mplu_zrenorm", "mplu_zconvert", "mplu_zgetrf_wsbytes", "mplu_zgetrf",
                 "mplu_zgetrs_wsbytes", "mplu_zgetrs", "mplu_zgesv_wsbytes", "mplu_zgesv",
                 "mplu_zgesv_noalloc",
                 "mplu_zgemm_wsbytes", "mplu_zgemm", "mplu_dgetrf_wsbytes", "mplu_dgetrf",
                 "mplu_dgetrs_wsbytes", "mplu_dgetrs", "mplu_dgesv_wsbytes", "mplu_dgesv",
                 "mplu_dgemm"):
        getattr(L, name).restype = ct.c_int
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().mplu_strerror(rc).decode()
        raise MPLUError(f"{what} failed with code {rc}: {msg}")


def _zmat(T: torch.Tensor) -> ZMat:
    if T.dtype != torch.float64 or T.dim() != 4 or T.shape[0] != 2:
        raise ValueError("expected a float64 tensor of shape (2, C, ncols, ld)")
    if not T.is_contiguous():
        raise ValueError("plane tensor must be contiguous")
    if not T.is_cuda:
        raise ValueError("plane tensor must live on the GPU")
    return ZMat(T.data_ptr(), T.shape[3], T.shape[2] * T.shape[3])


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


FLAG_NO_LOOKAHEAD = 1


FLAG_EXPIRE_WAITS = 2

# the look-ahead's second stream for each (device, caller stream): created by torch at the
# default priority on first use and kept, like torch's own stream pool
_aux_streams: dict = {}


def _aux_stream():
    cur = torch.cuda.current_stream()
    key = (cur.device.index, cur.cuda_stream)
    s = _aux_streams.get(key)
    if s is None:
        s = torch.cuda.Stream(device=cur.device)
        _aux_streams[key] = s
    return s.cuda_stream


def _opts(panel=64, method="3m", n_slices=0, slice_bits=0, lookahead=True, flags=0) -> Opts:
    m = _METHODS[method] if isinstance(method, str) else int(method)
    return Opts(int(panel), m, int(n_slices), int(slice_bits),
                int(flags) | (0 if lookahead else FLAG_NO_LOOKAHEAD),
                _aux_stream() if lookahead else None)


def _gemm_opts(method="3m", n_slices=0, slice_bits=0) -> Opts:
    m = _METHODS[method] if isinstance(method, str) else int(method)
    return Opts(64, m, int(n_slices), int(slice_bits), 0, None)


def _work(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def renorm_(A: torch.Tensor, m: int | None = None) -> torch.Tensor:
    """Make components non-overlapping, in place."""
    C = A.shape[1]
    m = A.shape[3] if m is None else m
    _check(lib().mplu_zrenorm(C, m, A.shape[2], _zmat(A), _stream()), "mplu_zrenorm")
    return A


def convert(A: torch.Tensor, Cout: int) -> torch.Tensor:
    """Copy of A with Cout components (widening is exact)."""
    C, ncols, ld = A.shape[1], A.shape[2], A.shape[3]
    B = torch.empty((2, Cout, ncols, ld), dtype=torch.float64, device=A.device)
    _check(lib().mplu_zconvert(C, Cout, ld, ncols, _zmat(A), _zmat(B), _stream()),
           "mplu_zconvert")
    return B


def getrf(A: torch.Tensor, panel: int = 64, method="3m", m: int | None = None,
          n_slices: int = 0, slice_bits: int = 0, work: torch.Tensor | None = None,
          lookahead: bool = True):
    """In-place P A = L U.  Returns (ipiv int32 device tensor, info int32 device tensor)."""
    C, n = A.shape[1], A.shape[2]
    m = A.shape[3] if m is None else m
    o = _opts(panel, method, n_slices, slice_bits, lookahead)
    nb = ct.c_size_t()
    _check(lib().mplu_zgetrf_wsbytes(C, m, n, ct.byref(o), ct.byref(nb)), "wsbytes")
    if work is None or work.numel() < nb.value:
        work = _work(nb.value, A.device)
    ipiv = torch.zeros(max(1, min(m, n)), dtype=torch.int32, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _check(lib().mplu_zgetrf(C, m, n, _zmat(A), ipiv.data_ptr(), info.data_ptr(), ct.byref(o),
                             work.data_ptr(), work.numel(), _stream()), "mplu_zgetrf")
    return ipiv[: min(m, n)], info


def getrs(LU: torch.Tensor, ipiv: torch.Tensor, B: torch.Tensor, trans: str = "N",
          work: torch.Tensor | None = None) -> torch.Tensor:
    """Solve A X = B ('N') or A^H X = B ('C') in place in B."""
    C, n = LU.shape[1], LU.shape[2]
    nrhs = B.shape[2]
    nb = ct.c_size_t()
    _check(lib().mplu_zgetrs_wsbytes(C, n, nrhs, ct.byref(nb)), "wsbytes")
    if work is None or work.numel() < nb.value:
        work = _work(nb.value, LU.device)
    ipiv = ipiv.to(torch.int32).contiguous()
    _check(lib().mplu_zgetrs(C, trans.encode(), n, nrhs, _zmat(LU), ipiv.data_ptr(), _zmat(B),
                             work.data_ptr(), work.numel(), _stream()), "mplu_zgetrs")
    return B


def gesv(A: torch.Tensor, B: torch.Tensor, panel: int = 64, method="3m", n_slices: int = 0,
         slice_bits: int = 0, work: torch.Tensor | None = None, lookahead: bool = True):
    """In place: A := factors, B := X.  Returns (ipiv, info)."""
    C, n = A.shape[1], A.shape[2]
    nrhs = B.shape[2]
    o = _opts(panel, method, n_slices, slice_bits, lookahead)
    nb = ct.c_size_t()
    _check(lib().mplu_zgesv_wsbytes(C, n, nrhs, ct.byref(o), ct.byref(nb)), "wsbytes")
    if work is None or work.numel() < nb.value:
        work = _work(nb.value, A.device)
    ipiv = torch.zeros(max(1, n), dtype=torch.int32, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _check(lib().mplu_zgesv(C, n, nrhs, _zmat(A), ipiv.data_ptr(), _zmat(B), info.data_ptr(),
                            ct.byref(o), work.data_ptr(), work.numel(), _stream()), "mplu_zgesv")
    return ipiv[:n], info


def gesv_noalloc(A: torch.Tensor, B: torch.Tensor, panel: int = 64, method="3m",
                 n_slices: int = 0, slice_bits: int = 0):
    """gesv without a workspace argument: the library's static scratch stands in for it
    (no device allocation by the library; the ipiv and info outputs are allocated here,
    callers that cannot allocate call mplu_zgesv_noalloc with their own).  Every step
    runs in order on the current stream.  Returns (ipiv, info)."""
    C, n = A.shape[1], A.shape[2]
    nrhs = B.shape[2]
    o = _opts(panel, method, n_slices, slice_bits, lookahead=False)
    ipiv = torch.zeros(max(1, n), dtype=torch.int32, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _check(lib().mplu_zgesv_noalloc(C, n, nrhs, _zmat(A), ipiv.data_ptr(), _zmat(B),
                                    info.data_ptr(), ct.byref(o), _stream()),
           "mplu_zgesv_noalloc")
    return ipiv[:n], info


def gemm(A: torch.Tensor, B: torch.Tensor, Cm: torch.Tensor | None = None, opA: str = "N",
         opB: str = "N", alpha: int = 1, method="3m", m: int | None = None,
         n: int | None = None, k: int | None = None, n_slices: int = 0,
         slice_bits: int = 0) -> torch.Tensor:
    """Cm := beta Cm + alpha op(A) op(B) (beta = 1 when Cm is given, else a new Cm)."""
    C = A.shape[1]
    if m is None:
        m = A.shape[3] if opA == "N" else A.shape[2]
    if k is None:
        k = A.shape[2] if opA == "N" else A.shape[3]
    if n is None:
        n = B.shape[2] if opB == "N" else B.shape[3]
    beta = 1
    if Cm is None:
        beta = 0
        Cm = torch.empty((2, C, n, m), dtype=torch.float64, device=A.device)
    meth = _METHODS[method] if isinstance(method, str) else int(method)
    o = _gemm_opts(meth, n_slices, slice_bits)
    nb = ct.c_size_t()
    _check(lib().mplu_zgemm_wsbytes(C, m, n, k, meth, ct.byref(o), ct.byref(nb)), "wsbytes")
    work = _work(nb.value, A.device)
    _check(lib().mplu_zgemm(C, opA.encode(), opB.encode(), m, n, k, int(alpha), _zmat(A),
                            _zmat(B), beta, _zmat(Cm), meth, ct.byref(o), work.data_ptr(),
                            work.numel(), _stream()), "mplu_zgemm")
    return Cm


# ---------------------------------------------------------------- real matrices
# float64 CUDA tensors of shape (C, ncols, ld): plane [c] is component c, column-major,
# so element (i, j) is T[c, j, i].

def _dmat(T: torch.Tensor) -> DMat:
    if T.dtype != torch.float64 or T.dim() != 3:
        raise ValueError("expected a float64 tensor of shape (C, ncols, ld)")
    if not T.is_contiguous():
        raise ValueError("plane tensor must be contiguous")
    if not T.is_cuda:
        raise ValueError("plane tensor must live on the GPU")
    return DMat(T.data_ptr(), T.shape[2], T.shape[1] * T.shape[2])


def dgetrf(A: torch.Tensor, panel: int = 64, method="3m", m: int | None = None,
           work: torch.Tensor | None = None, lookahead: bool = True):
    """In-place P A = L U of a real matrix ('3m' / '4m' select the real product, the split
    methods split real operands).  Returns (ipiv, info) int32 device tensors."""
    C, n = A.shape[0], A.shape[1]
    m = A.shape[2] if m is None else m
    o = _opts(panel, method, 0, 0, lookahead)
    nb = ct.c_size_t()
    _check(lib().mplu_dgetrf_wsbytes(C, m, n, ct.byref(o), ct.byref(nb)), "wsbytes")
    if work is None or work.numel() < nb.value:
        work = _work(nb.value, A.device)
    ipiv = torch.zeros(max(1, min(m, n)), dtype=torch.int32, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _check(lib().mplu_dgetrf(C, m, n, _dmat(A), ipiv.data_ptr(), info.data_ptr(), ct.byref(o),
                             work.data_ptr(), work.numel(), _stream()), "mplu_dgetrf")
    return ipiv[: min(m, n)], info


def dgetrs(LU: torch.Tensor, ipiv: torch.Tensor, B: torch.Tensor, trans: str = "N",
           work: torch.Tensor | None = None) -> torch.Tensor:
    """Solve A X = B ('N') or A^T X = B ('T') in place in B (real)."""
    C, n = LU.shape[0], LU.shape[1]
    nrhs = B.shape[1]
    nb = ct.c_size_t()
    _check(lib().mplu_dgetrs_wsbytes(C, n, nrhs, ct.byref(nb)), "wsbytes")
    if work is None or work.numel() < nb.value:
        work = _work(nb.value, LU.device)
    ipiv = ipiv.to(torch.int32).contiguous()
    _check(lib().mplu_dgetrs(C, trans.encode(), n, nrhs, _dmat(LU), ipiv.data_ptr(), _dmat(B),
                             work.data_ptr(), work.numel(), _stream()), "mplu_dgetrs")
    return B


def dgesv(A: torch.Tensor, B: torch.Tensor, panel: int = 64, method="3m",
          work: torch.Tensor | None = None, lookahead: bool = True):
    """Real A X = B in place: A := factors, B := X.  Returns (ipiv, info)."""
    C, n = A.shape[0], A.shape[1]
    nrhs = B.shape[1]
    o = _opts(panel, method, 0, 0, lookahead)
    nb = ct.c_size_t()
    _check(lib().mplu_dgesv_wsbytes(C, n, nrhs, ct.byref(o), ct.byref(nb)), "wsbytes")
    if work is None or work.numel() < nb.value:
        work = _work(nb.value, A.device)
    ipiv = torch.zeros(max(1, n), dtype=torch.int32, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _check(lib().mplu_dgesv(C, n, nrhs, _dmat(A), ipiv.data_ptr(), _dmat(B), info.data_ptr(),
                            ct.byref(o), work.data_ptr(), work.numel(), _stream()), "mplu_dgesv")
    return ipiv[:n], info


def dgemm(A: torch.Tensor, B: torch.Tensor, Cm: torch.Tensor | None = None, opA: str = "N",
          opB: str = "N", alpha: int = 1) -> torch.Tensor:
    """Cm := beta Cm + alpha op(A) op(B) for real matrices (beta = 1 when Cm is given)."""
    C = A.shape[0]
    m = A.shape[2] if opA == "N" else A.shape[1]
    k = A.shape[1] if opA == "N" else A.shape[2]
    n = B.shape[1] if opB == "N" else B.shape[2]
    beta = 1
    if Cm is None:
        beta = 0
        Cm = torch.empty((C, n, m), dtype=torch.float64, device=A.device)
    _check(lib().mplu_dgemm(C, opA.encode(), opB.encode(), m, n, k, int(alpha), _dmat(A),
                            _dmat(B), beta, _dmat(Cm), _stream()), "mplu_dgemm")
    return Cm


from .autograd import lu_factor, lu_solve, solve  # noqa: E402  (needs the functions above)
