/*
 * mplu.h -- complex multi-component (double-double / triple-double / quadruple-double)
 * LU factorisation with partial pivoting and linear solves on AMD Instinct MI355X (gfx950).
 *
 * The method is the blocked right-looking LU of Kouya, "Performance evaluation of
 * accelerated complex multiple-precision LU decomposition" (Sec. 3, Eq. linear_eq):
 * factor a K-column panel with partial pivoting, apply its row interchanges, solve for
 * the block row of U, then update the trailing matrix A22 -= L21 U12 with a complex
 * multiple-precision matrix product computed by the 4M method (Eq. 4m), the 3M method
 * (Eq. 3m_cemm) or an error-free split of the operands whose slice products are exact
 * on the matrix cores (the Ozaki scheme of Sec. 2.3).
 *
 * NUMBER FORMAT (Sec. 1, Sec. 2.2 and Fig. 1).  A real value is an unevaluated sum of
 * C binary64 components (C = 2, 3, 4: 106, 159, 212 bits).  A complex matrix keeps its
 * real and imaginary parts apart: it is 2*C planes of binary64,
 *     plane q = ri*C + c   (ri = 0 real part, ri = 1 imaginary part; c = component)
 * at  planes + q*plane_stride, each plane column-major: element (i, j) at [j*ld + i].
 * Components should be non-overlapping (|c_{k+1}| <= ulp(c_k)/2); mplu_zrenorm makes
 * them so, and every routine accepts any finite components.
 *
 * CONVENTIONS SHARED BY ALL ENTRY POINTS
 *  - Pointers named d_* and every mplu_zmat_t.planes are DEVICE pointers (hipMalloc'd or
 *    from a caching allocator).  The caller owns all memory and streams; the library
 *    never allocates device memory, frees or synchronises the host, and keeps no state
 *    between calls other than cached device properties (and the static scratch of
 *    mplu_zgesv_noalloc).  Work is enqueued on `stream` (a hipStream_t; NULL = default);
 *    mplu_zgetrf also forks part of it onto the caller's opts->aux_stream, if given, and
 *    joins it back (see there).
 *  - Return value (synchronous, decided before anything is enqueued): 0 on success,
 *    -i when argument i (1-based) is invalid, or one of the MPLU_E_* codes below.
 *  - Numerical failure is reported asynchronously through d_info (LAPACK getf2 rules).
 *  - NaN and infinity are not checked; they propagate.
 *  - Every entry point is re-entrant; calls on different streams may run concurrently
 *    provided they use different workspaces.
 */
#ifndef MPLU_H
#define MPLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of binary64 components (Sec. 1). */
typedef enum { MPLU_DD = 2, MPLU_TD = 3, MPLU_QD = 4 } mplu_prec_t;

/* Trailing-update product. */
typedef enum {
  MPLU_GEMM_4M = 0,        /* Eq. 4m: four real products                                */
  MPLU_GEMM_3M = 1,        /* Eq. 3m_cemm: three real products plus additions           */
  MPLU_GEMM_SPLIT_F64 = 2, /* Sec. 2.3 Ozaki scheme: exact slice products on FP64 MFMA  */
  MPLU_GEMM_SPLIT_I8 = 3,  /* same split with 7-bit INT8 slices, exact INT32 sums       */
  MPLU_GEMM_STRASSEN = 4   /* one level of Winograd's variant of Strassen's algorithm
                              over 3M products (Sec. 2.1): mplu_zgemm ('N', 'N') and the
                              trailing updates of the complex mplu_zgetrf / mplu_zgesv
                              (the Strassen LU of Sec. 3 / Table 1)                      */
} mplu_gemm_t;

/* A complex multi-component matrix: see NUMBER FORMAT above. */
typedef struct {
  double *planes;
  int64_t ld;           /* >= max(1, rows)                                   */
  int64_t plane_stride; /* >= ld * cols; distance between planes in doubles  */
} mplu_zmat_t;

/* Options; a NULL pointer selects the defaults given in brackets. */
typedef struct {
  int32_t panel;      /* panel width K (= NDIM of Sec. 3) [64], at most 128 (the panel is
                         held in LDS); >= min(m, n) gives the unblocked LU, which therefore
                         needs min(m, n) <= 128; an effective width min(panel, min(m, n))
                         above 128 makes mplu_zgetrf return MPLU_E_UNSUPPORTED          */
  int32_t gemm;       /* mplu_gemm_t for the trailing update [MPLU_GEMM_3M]; with
                         MPLU_GEMM_STRASSEN the look-ahead's narrow product of the next
                         panel's columns stays plain 3M                                   */
  int32_t n_slices;   /* split methods: slices per operand, 0 = automatic                   */
  int32_t slice_bits; /* split methods: bits per slice, 0 = automatic                       */
  int32_t flags;      /* MPLU_FLAG_* bits [0]                                               */
  void *aux_stream;   /* mplu_zgetrf / mplu_zgesv: a second hipStream_t of the caller's on
                         the same device, for the look-ahead described under mplu_zgetrf
                         [NULL: no look-ahead, every step in order on `stream`]          */
} mplu_opts_t;

/* mplu_zgetrf / mplu_zgesv flag: run every step on `stream` in order, without the
 * look-ahead, even when aux_stream is given.  The results are bitwise the same. */
#define MPLU_FLAG_NO_LOOKAHEAD 1
/* mplu_zgetrf / mplu_zgesv flag, for tests of the failure path only: the panel's bounded
 * inter-workgroup waits start out expired, so each gives up at its first look at the
 * expiry word (every kernel still ends normally); *d_info then reads
 * MPLU_INFO_SYNC_TIMEOUT and the factors are not to be used. */
#define MPLU_FLAG_EXPIRE_WAITS 2

/* Error codes (besides -i for argument i). */
#define MPLU_OK 0
#define MPLU_E_WORKSPACE (-100)   /* work_bytes below the *_wsbytes figure            */
#define MPLU_E_HIP (-101)         /* a HIP runtime call or kernel launch failed       */
#define MPLU_E_UNSUPPORTED (-102) /* size / option combination not supported          */
#define MPLU_E_SCRATCH (-103)     /* mplu_zgesv_noalloc: workspace need above its scratch */

/* Value written to *d_info when the panel's inter-workgroup barrier did not complete
 * within its bounded wait (the factors are then invalid). */
#define MPLU_INFO_SYNC_TIMEOUT (-9999)

/*
 * mplu_zrenorm -- make the components of every element non-overlapping, in place
 * (storage step of the method: Sec. 2.2 keeps values as unevaluated component sums).
 *   prec: C; m, n: rows, cols (>= 0); A: matrix, modified in place.
 */
int mplu_zrenorm(int prec, int64_t m, int64_t n, mplu_zmat_t A, void *stream);

/*
 * mplu_zconvert -- B := A converted from prec_src to prec_dst components (widening pads
 * with zeros and is exact; narrowing rounds to the nearer representable sum).
 * A and B must not overlap.
 */
int mplu_zconvert(int prec_src, int prec_dst, int64_t m, int64_t n, mplu_zmat_t A,
                  mplu_zmat_t B, void *stream);

/*
 * mplu_zgetrf_wsbytes -- workspace bytes mplu_zgetrf needs for these sizes and options.
 */
int mplu_zgetrf_wsbytes(int prec, int64_t m, int64_t n, const mplu_opts_t *opts,
                        size_t *bytes);

/*
 * mplu_zgetrf -- P A = L U by blocked right-looking LU with partial pivoting (Sec. 3,
 * Fig. 8; "Normal LU" when opts->panel >= min(m, n)).
 *   Look-ahead (when opts->aux_stream is given): while panel k+1 is factored on
 *   `stream`, the step-k update of the columns right of panel k+1 runs on aux_stream,
 *   forked from and joined back to `stream` with three events that the call creates and
 *   releases, so the call still behaves as one ordered unit of work on `stream` (also
 *   under stream capture): aux_stream starts after the work already on `stream`, and
 *   work enqueued on `stream` after the call starts after all of it.  Calls on different
 *   caller streams with different aux streams proceed independently.  Without
 *   aux_stream, or with MPLU_FLAG_NO_LOOKAHEAD, every step runs in order on `stream`.
 *   A (m x n) is overwritten by L (unit diagonal not stored) and U.
 *   d_ipiv: min(m,n) int32, 1-based row interchanges in LAPACK order (row k was swapped
 *           with row d_ipiv[k]-1, for k ascending).
 *   d_info: one int32: 0, or k (1-based) for the first exactly-zero pivot (that column is
 *           neither swapped nor scaled and the factorisation goes on), or
 *           MPLU_INFO_SYNC_TIMEOUT.
 *   Pivot choice: the row maximising |Re| + |Im| in full precision, the lowest row on ties.
 *   d_work: at least mplu_zgetrf_wsbytes bytes of device memory, 256-byte aligned.
 */
int mplu_zgetrf(int prec, int64_t m, int64_t n, mplu_zmat_t A, int32_t *d_ipiv,
                int32_t *d_info, const mplu_opts_t *opts, void *d_work, size_t work_bytes,
                void *stream);

/* mplu_zgetrs_wsbytes -- workspace bytes mplu_zgetrs needs. */
int mplu_zgetrs_wsbytes(int prec, int64_t n, int64_t nrhs, size_t *bytes);

/*
 * mplu_zgetrs -- solve A X = B (trans 'N') or A^H X = B (trans 'C') with the factors of
 * mplu_zgetrf: row interchanges, then forward and backward substitution (Sec. 4).
 *   LU, d_ipiv: output of mplu_zgetrf for an n x n A.  B: n x nrhs, overwritten by X.
 */
int mplu_zgetrs(int prec, char trans, int64_t n, int64_t nrhs, mplu_zmat_t LU,
                const int32_t *d_ipiv, mplu_zmat_t B, void *d_work, size_t work_bytes,
                void *stream);

/* mplu_zgesv_wsbytes -- workspace bytes mplu_zgesv needs. */
int mplu_zgesv_wsbytes(int prec, int64_t n, int64_t nrhs, const mplu_opts_t *opts,
                       size_t *bytes);

/*
 * mplu_zgesv -- solve A X = B: mplu_zgetrf followed by mplu_zgetrs('N') (Eq. linear_eq).
 *   A (n x n) is overwritten by its factors, B (n x nrhs) by X.  If the factorisation
 *   finds an exactly-zero pivot, X holds non-finite values and *d_info > 0.
 */
int mplu_zgesv(int prec, int64_t n, int64_t nrhs, mplu_zmat_t A, int32_t *d_ipiv,
               mplu_zmat_t B, int32_t *d_info, const mplu_opts_t *opts, void *d_work,
               size_t work_bytes, void *stream);

/*
 * mplu_zgesv_noalloc -- mplu_zgesv for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 *   Same arguments, results and d_info as mplu_zgesv (bitwise the same X, factors and
 *   pivots), without d_work / work_bytes: the workspace is a static device array of
 *   MPLU_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the process
 *   ends and looked up on the first call on each device.  The call allocates nothing,
 *   creates no stream or event, and runs every step in order on `stream` (the look-ahead
 *   of mplu_zgetrf needs a second stream, so it is not used; MPLU_FLAG_NO_LOOKAHEAD is
 *   implied).
 *   Returns MPLU_E_SCRATCH, before enqueuing anything, when mplu_zgesv_wsbytes for these
 *   sizes and options exceeds MPLU_NOALLOC_SCRATCH_BYTES (e.g. QD with panel 128 fits for
 *   n*nrhs up to about 3.8e5 complex entries of B per call; the split methods' digit
 *   planes fit only small n).
 *   All calls on one GPU share its scratch array: calls that overlap in time on one GPU
 *   (different streams or threads) race and must be serialised by the caller.  Each
 *   call clears what it needs zeroed itself; nothing is carried between calls.
 */
#define MPLU_NOALLOC_SCRATCH_BYTES (16u << 20)
int mplu_zgesv_noalloc(int prec, int64_t n, int64_t nrhs, mplu_zmat_t A, int32_t *d_ipiv,
                       mplu_zmat_t B, int32_t *d_info, const mplu_opts_t *opts,
                       void *stream);

/* mplu_zgemm_wsbytes -- workspace bytes mplu_zgemm needs (0 for 3M and 4M; the split
 * digit planes; for MPLU_GEMM_STRASSEN an m x n product and the two half-size operand
 * sums, complex). */
int mplu_zgemm_wsbytes(int prec, int64_t m, int64_t n, int64_t k, int method,
                       const mplu_opts_t *opts, size_t *bytes);

/*
 * mplu_zgemm -- Cm := beta*Cm + alpha*op(A)*op(B), the complex multiple-precision matrix
 * product of Sec. 2.1 (Eq. 4m / Eq. 3m_cemm) or its split form (Sec. 2.3).
 *   opA, opB: 'N', 'T' or 'C' (conjugate transpose).  op(A) is m x k, op(B) is k x n.
 *   alpha_sign: +1 or -1.  beta: 0 (Cm is overwritten) or 1 (Cm is accumulated into).
 *   method: mplu_gemm_t.  Cm must not overlap A or B.  MPLU_GEMM_STRASSEN takes
 *   opA = opB = 'N' only (MPLU_E_UNSUPPORTED otherwise); its error bound is normwise
 *   (Strassen-type), not elementwise like the other forms.  mplu_zgetrf rejects it.
 */
int mplu_zgemm(int prec, char opA, char opB, int64_t m, int64_t n, int64_t k,
               int alpha_sign, mplu_zmat_t A, mplu_zmat_t B, int beta, mplu_zmat_t Cm,
               int method, const mplu_opts_t *opts, void *d_work, size_t work_bytes,
               void *stream);

/*
 * REAL MATRICES -- the Im = 0 case of the same method (the paper's earlier real DD / TD /
 * QD LU that Sec. 1 builds on; Sec. 3 with every imaginary part zero).
 *
 * A real multi-component matrix is C planes: plane c (component c) at
 * planes + c*plane_stride, each column-major (element (i, j) at [j*ld + i]).
 *
 * mplu_dgetrf / mplu_dgetrs / mplu_dgesv run the real variants of the complex kernels on
 * the caller's C planes: the panel (pivot measure |a| in full precision, real
 * reciprocal), interchanges, triangular solves and substitutions, and the real product
 * (only T1 = Re(L21) Re(U12) of Eq. 3m_cemm) for the trailing and block updates.
 * opts->gemm: MPLU_GEMM_4M and MPLU_GEMM_3M both select the real product; the split
 * methods split the real operands (one real product of digit pairs instead of three);
 * MPLU_GEMM_STRASSEN is complex only (MPLU_E_UNSUPPORTED).
 * Argument meaning, pivots, d_info, ownership, errors and workspace sizes are as for the
 * complex routines.
 */
typedef struct {
  double *planes;
  int64_t ld;           /* >= max(1, rows)                                   */
  int64_t plane_stride; /* >= ld * cols; distance between planes in doubles  */
} mplu_dmat_t;

/* mplu_dgetrf_wsbytes -- workspace bytes mplu_dgetrf needs. */
int mplu_dgetrf_wsbytes(int prec, int64_t m, int64_t n, const mplu_opts_t *opts,
                        size_t *bytes);

/* mplu_dgetrf -- P A = L U of a real m x n A (see mplu_zgetrf). */
int mplu_dgetrf(int prec, int64_t m, int64_t n, mplu_dmat_t A, int32_t *d_ipiv,
                int32_t *d_info, const mplu_opts_t *opts, void *d_work, size_t work_bytes,
                void *stream);

/* mplu_dgetrs_wsbytes -- workspace bytes mplu_dgetrs needs. */
int mplu_dgetrs_wsbytes(int prec, int64_t n, int64_t nrhs, size_t *bytes);

/* mplu_dgetrs -- solve A X = B (trans 'N') or A^T X = B (trans 'T') with the factors of
 * mplu_dgetrf (Sec. 4).  B (n x nrhs) is overwritten by X. */
int mplu_dgetrs(int prec, char trans, int64_t n, int64_t nrhs, mplu_dmat_t LU,
                const int32_t *d_ipiv, mplu_dmat_t B, void *d_work, size_t work_bytes,
                void *stream);

/* mplu_dgesv_wsbytes -- workspace bytes mplu_dgesv needs. */
int mplu_dgesv_wsbytes(int prec, int64_t n, int64_t nrhs, const mplu_opts_t *opts,
                       size_t *bytes);

/* mplu_dgesv -- solve the real system A X = B: mplu_dgetrf then mplu_dgetrs('N').
 *   A (n x n) is overwritten by its factors, B (n x nrhs) by X. */
int mplu_dgesv(int prec, int64_t n, int64_t nrhs, mplu_dmat_t A, int32_t *d_ipiv,
               mplu_dmat_t B, int32_t *d_info, const mplu_opts_t *opts, void *d_work,
               size_t work_bytes, void *stream);

/*
 * mplu_dgemm -- Cm := beta*Cm + alpha*op(A)*op(B) for real multi-component matrices, the
 * real product the factorisation's trailing update uses (no workspace).
 *   opA, opB: 'N' or 'T'.  alpha_sign: +1 or -1.  beta: 0 or 1.  Cm must not overlap A
 *   or B.
 */
int mplu_dgemm(int prec, char opA, char opB, int64_t m, int64_t n, int64_t k,
               int alpha_sign, mplu_dmat_t A, mplu_dmat_t B, int beta, mplu_dmat_t Cm,
               void *stream);

/* mplu_strerror -- static text for a return code. */
const char *mplu_strerror(int code);

/* mplu_version -- library version number (major*10000 + minor*100 + patch). */
int mplu_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPLU_H */
