// capi.cpp -- the exported C ABI (declared in include/mplu.h): argument checks, workspace
// layout and the host-side loops of the blocked LU (Kouya Sec. 3, Fig. 8) and of the
// forward / backward substitutions (Sec. 4).  All work is enqueued on the caller's
// stream (and, for the factorisation's look-ahead, on the second stream the caller
// passes in the options); nothing here allocates device memory, frees or synchronises.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "mplu.h"
#include "common.hpp"

using namespace mplu;

namespace {

constexpr int kDefaultPanel = 64;
constexpr int kMaxPanel = 128;
constexpr int kSolveBlock = 64;

inline bool prec_ok(int p) { return p == 2 || p == 3 || p == 4; }

// 0 if the matrix descriptor is usable for rows x cols
inline bool mat_ok(const mplu_zmat_t &A, int64_t rows, int64_t cols) {
  if (rows < 0 || cols < 0) return false;
  if (rows == 0 || cols == 0) return true;
  if (A.planes == nullptr) return false;
  if (A.ld < (rows > 1 ? rows : 1)) return false;
  if (A.plane_stride < A.ld * cols) return false;
  return true;
}

inline ZM zm(const mplu_zmat_t &A) { return ZM{A.planes, A.ld, A.plane_stride}; }

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int panel_width(const mplu_opts_t *o) {
  int kb = (o && o->panel > 0) ? o->panel : kDefaultPanel;
  return kb > kMaxPanel ? kMaxPanel : kb;
}

inline int gemm_method(const mplu_opts_t *o) { return o ? o->gemm : MPLU_GEMM_3M; }

// internal trailing-update method of the real factorisation: the real product (the
// Im = 0 case of Eq. 3m_cemm) on the real planes only
constexpr int kGemmReal = 100;

#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return MPLU_E_HIP; \
  } while (0)

// right-hand-side counts up to this use the one-launch substitutions (k_trsv), larger
// ones the blocked sweep of triangular solves and products
constexpr int64_t kSvMaxRhs = 32;

int getrs_ws(int C, int64_t n, int64_t nrhs, size_t *bytes) {
  *bytes = align256(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)) +
           align256(sizeof(double) * 2 * C * (size_t)(n > 0 ? n : 1) * (size_t)(nrhs > 0 ? nrhs : 1)) +
           align256(sizeof(int32_t) * (size_t)trsv_flag_words(n, nrhs < kSvMaxRhs ? nrhs : kSvMaxRhs));
  return 0;
}

inline bool is_split(int method) {
  return method == MPLU_GEMM_SPLIT_F64 || method == MPLU_GEMM_SPLIT_I8;
}

// one Winograd level over 3M products (defined below with its workspace layout)
size_t strassen_ws(int C, int64_t m, int64_t n, int64_t k);
hipError_t strassen_zgemm(int C, int64_t m, int64_t n, int64_t k, int alpha, ZM A, ZM B,
                          int beta, ZM Cm, void *ws, hipStream_t s);

// slice options: n_slices 0 = default; slice_bits 0 or the fixed digit width (7 for INT8,
// 22 for FP64)
inline bool split_opts_ok(int C, int method, const mplu_opts_t *o) {
  if (!is_split(method)) return true;
  const bool i8 = method == MPLU_GEMM_SPLIT_I8;
  const int S = o ? o->n_slices : 0;
  const int w = o ? o->slice_bits : 0;
  if (w != 0 && w != (i8 ? 7 : 22)) return false;
  return split_supported(C, i8, S);
}

// getrf workspace: three panel workspaces (consecutive panels rotate through them, so the
// step-k interchanges stay readable until the second stream has applied them to the
// columns left of the panel), then for the split methods one slice workspace for the rest
// of the trailing matrix and one for the next panel's columns
struct GetrfWS {
  size_t panel, split_rest, split_next, total;
};

GetrfWS getrf_layout(int C, int64_t m, int64_t n, const mplu_opts_t *o) {
  const int64_t mn = m < n ? m : n;
  int kb = panel_width(o);
  if (mn > 0 && kb > mn) kb = (int)mn;
  if (kb < 1) kb = 1;
  GetrfWS w{};
  w.panel = align256(panel_ws_bytes(C, kb));
  const int method = gemm_method(o);
  if (is_split(method)) {
    const bool i8 = method == MPLU_GEMM_SPLIT_I8;
    const int S = o ? o->n_slices : 0;
    w.split_rest = align256(split_ws_bytes(C, i8, m, n, kb, S));
    w.split_next = align256(split_ws_bytes(C, i8, m, kb, kb, S));
  } else if (method == MPLU_GEMM_STRASSEN) {
    // the rest of the trailing matrix (the next panel's columns use plain 3M)
    w.split_rest = align256(strassen_ws(C, m, n, kb));
  }
  w.total = 3 * w.panel + w.split_rest + w.split_next;
  return w;
}

int getrf_ws(int C, int64_t m, int64_t n, const mplu_opts_t *o, size_t *bytes) {
  *bytes = getrf_layout(C, m, n, o).total;
  return 0;
}

// The look-ahead's ordering events: created per call (they are tied to the caller's two
// streams, which may change from call to call) and released at its end; a release while
// work that records or waits on them is still queued takes effect once that work is done.
struct LookaheadEvents {
  hipEvent_t panel = nullptr, rest = nullptr, chain = nullptr;
  hipError_t create() {
    hipError_t e;
    if ((e = hipEventCreateWithFlags(&panel, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&rest, hipEventDisableTiming)) != hipSuccess) return e;
    return hipEventCreateWithFlags(&chain, hipEventDisableTiming);
  }
  ~LookaheadEvents() {
    if (panel) (void)hipEventDestroy(panel);
    if (rest) (void)hipEventDestroy(rest);
    if (chain) (void)hipEventDestroy(chain);
  }
};

// the trailing update of one step restricted to columns [c0, c1): U12 := L11^-1 A12 on
// those columns, then A22 -= L21 U12 on them
// urgent: the next panel's columns, on the critical path of the look-ahead schedule
hipError_t step_trsm(int C, ZM a, int64_t j, int jb, int64_t c0, int64_t c1, hipStream_t s,
                     const int32_t *swl, bool real, bool urgent = false) {
  if (c1 <= c0) return hipSuccess;
  return launch_trsm(C, true, true, false, a, j, jb, a, j, c0, c1 - c0, s, swl, 2 * jb, real,
                     urgent);
}

// real: a real matrix (the split methods then split real operands; the others use the
// real product)
hipError_t step_gemm(int C, int method, int S, ZM a, int64_t m, int64_t j, int jb, int64_t c0,
                     int64_t c1, void *split_ws, hipStream_t s, bool real, bool urgent = false) {
  if (c1 <= c0 || j + jb >= m) return hipSuccess;
  if (method == MPLU_GEMM_STRASSEN)  // complex only (getrf_core rejects it for real)
    return strassen_zgemm(C, m - j - jb, c1 - c0, jb, -1, ZM{a.p + j * a.ld + j + jb, a.ld, a.ps},
                          ZM{a.p + c0 * a.ld + j, a.ld, a.ps},
                          1, ZM{a.p + c0 * a.ld + j + jb, a.ld, a.ps}, split_ws, s);
  if (is_split(method))
    return launch_gemm_split(C, method == MPLU_GEMM_SPLIT_I8, S, 'N', 'N', m - j - jb, c1 - c0,
                             jb, -1, a, j + jb, j, a, j, c0, 1, a, j + jb, c0, split_ws, s,
                             real);
  if (real) method = kGemmReal;
  return launch_gemm(C, method == kGemmReal ? 2 : (method == MPLU_GEMM_3M ? 1 : 0), 'N', 'N',
                     m - j - jb, c1 - c0, jb, -1, a, j + jb, j, a, j, c0, 1, a, j + jb, c0, s,
                     urgent);
}

hipError_t step_update(int C, int method, int S, ZM a, int64_t m, int64_t j, int jb, int64_t c0,
                       int64_t c1, void *split_ws, hipStream_t s, bool real) {
  hipError_t e = step_trsm(C, a, j, jb, c0, c1, s, nullptr, real);
  if (e != hipSuccess) return e;
  return step_gemm(C, method, S, a, m, j, jb, c0, c1, split_ws, s, real);
}

// ------------------------------------------------------------------ Strassen-Winograd
// C := beta C + alpha A B ('N', 'N') by one level of Winograd's variant of Strassen's
// algorithm (the paper's other fast product, Sec. 2.1) over 3M products: seven half-size
// complex products and fifteen matrix sums instead of eight products.  One level only:
// at the sizes this GPU runs, the half-size products still fill the device, quarter-size
// ones would not.  Odd sizes are peeled: the even leading part goes through the
// recursion and the last row, column and k term are plain 3M products.
//
// Workspace: W (m x n, the product), X (m/2 x k/2), Y (k/2 x n/2), complex.

inline ZM zsub(ZM a, int64_t i, int64_t j) { return ZM{a.p + j * a.ld + i, a.ld, a.ps}; }

inline size_t zmat_bytes(int C, int64_t r, int64_t c) {
  return align256(sizeof(double) * 2 * (size_t)C * (size_t)(r > 1 ? r : 1) * (size_t)(c > 0 ? c : 0));
}

size_t strassen_ws(int C, int64_t m, int64_t n, int64_t k) {
  return zmat_bytes(C, m, n) + zmat_bytes(C, m / 2, k / 2) + zmat_bytes(C, k / 2, n / 2);
}

// product on sub-blocks: O := beta O + alpha A B (3M)
inline hipError_t g3m(int C, int64_t m, int64_t n, int64_t k, int alpha, ZM A, ZM B, int beta,
                      ZM O, hipStream_t s) {
  return launch_gemm(C, 1, 'N', 'N', m, n, k, alpha, A, 0, 0, B, 0, 0, beta, O, 0, 0, s);
}

hipError_t strassen_zgemm(int C, int64_t m, int64_t n, int64_t k, int alpha, ZM A, ZM B,
                          int beta, ZM Cm, void *ws, hipStream_t s) {
  if (m == 0 || n == 0) return hipSuccess;
  char *wb = (char *)ws;
  const int64_t ldw = m > 1 ? m : 1;
  const ZM W{(double *)wb, ldw, ldw * n};
  const int64_t h = m / 2, q = n / 2, r = k / 2;  // half sizes
  const ZM X{(double *)(wb + zmat_bytes(C, m, n)), h > 1 ? h : 1, (h > 1 ? h : 1) * r};
  const ZM Y{(double *)(wb + zmat_bytes(C, m, n) + zmat_bytes(C, h, r)), r > 1 ? r : 1,
             (r > 1 ? r : 1) * q};
  hipError_t e;
#define GO(x)                              \
  do {                                     \
    if ((e = (x)) != hipSuccess) return e; \
  } while (0)
  if (h > 0 && q > 0 && r > 0) {
    const ZM A11 = A, A12 = zsub(A, 0, r), A21 = zsub(A, h, 0), A22 = zsub(A, h, r);
    const ZM B11 = B, B12 = zsub(B, 0, q), B21 = zsub(B, r, 0), B22 = zsub(B, r, q);
    const ZM W11 = W, W12 = zsub(W, 0, q), W21 = zsub(W, h, 0), W22 = zsub(W, h, q);
    GO(launch_zaxpby(C, h, r, 1, A11, -1, A21, X, s));     // X = S3 = A11 - A21
    GO(launch_zaxpby(C, r, q, 1, B22, -1, B12, Y, s));     // Y = T3 = B22 - B12
    GO(g3m(C, h, q, r, 1, X, Y, 0, W21, s));               // W21 = P7 = S3 T3
    GO(launch_zaxpby(C, h, r, 1, A21, 1, A22, X, s));      // X = S1 = A21 + A22
    GO(launch_zaxpby(C, r, q, 1, B12, -1, B11, Y, s));     // Y = T1 = B12 - B11
    GO(g3m(C, h, q, r, 1, X, Y, 0, W22, s));               // W22 = P5 = S1 T1
    GO(launch_zaxpby(C, h, r, 1, X, -1, A11, X, s));       // X = S2 = S1 - A11
    GO(launch_zaxpby(C, r, q, 1, B22, -1, Y, Y, s));       // Y = T2 = B22 - T1
    GO(g3m(C, h, q, r, 1, X, Y, 0, W12, s));               // W12 = P6 = S2 T2
    GO(launch_zaxpby(C, h, r, 1, A12, -1, X, X, s));       // X = S4 = A12 - S2
    GO(g3m(C, h, q, r, 1, A11, B11, 0, W11, s));           // W11 = P1 = A11 B11
    GO(launch_zaxpby(C, h, q, 1, W12, 1, W11, W12, s));    // W12 = U2 = P6 + P1
    GO(launch_zaxpby(C, h, q, 1, W21, 1, W12, W21, s));    // W21 = U3 = P7 + U2
    GO(launch_zaxpby(C, h, q, 1, W12, 1, W22, W12, s));    // W12 = U4 = U2 + P5
    GO(launch_zaxpby(C, h, q, 1, W22, 1, W21, W22, s));    // W22 = C22 = P5 + U3
    GO(g3m(C, h, q, r, 1, X, B22, 1, W12, s));             // W12 = C12 = U4 + S4 B22
    GO(launch_zaxpby(C, r, q, 1, Y, -1, B21, Y, s));       // Y = T4 = T2 - B21
    GO(g3m(C, h, q, r, -1, A22, Y, 1, W21, s));            // W21 = C21 = U3 - A22 T4
    GO(g3m(C, h, q, r, 1, A12, B21, 1, W11, s));           // W11 = C11 = P1 + A12 B21
    if (k % 2)  // the last k term of the even leading part
      GO(g3m(C, 2 * h, 2 * q, 1, 1, zsub(A, 0, k - 1), zsub(B, k - 1, 0), 1, W, s));
  } else if (h > 0 && q > 0) {  // k < 2: a plain product of the even leading part
    GO(g3m(C, 2 * h, 2 * q, k, 1, A, B, 0, W, s));
  }
  if (n % 2)  // last column, all rows
    GO(g3m(C, m, 1, k, 1, A, zsub(B, 0, n - 1), 0, zsub(W, 0, n - 1), s));
  if (m % 2 && q > 0)  // last row, the even leading columns
    GO(g3m(C, 1, 2 * q, k, 1, zsub(A, m - 1, 0), B, 0, zsub(W, m - 1, 0), s));
  // C := beta C + alpha W
  GO(launch_zaxpby(C, m, n, beta, Cm, alpha, W, Cm, s));
#undef GO
  return hipSuccess;
}

}  // namespace

extern "C" {

int mplu_version(void) { return 10100; }

const char *mplu_strerror(int code) {
  switch (code) {
    case MPLU_OK: return "success";
    case MPLU_E_WORKSPACE: return "workspace too small";
    case MPLU_E_HIP: return "HIP runtime error or kernel launch failure";
    case MPLU_E_UNSUPPORTED: return "unsupported size or option combination";
    case MPLU_E_SCRATCH:
      return "workspace need exceeds the static scratch of mplu_zgesv_noalloc "
             "(MPLU_NOALLOC_SCRATCH_BYTES)";
    default: break;
  }
  if (code < 0 && code > -20) return "invalid argument";
  return "unknown error";
}

int mplu_zrenorm(int prec, int64_t m, int64_t n, mplu_zmat_t A, void *stream) {
  if (!prec_ok(prec)) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!mat_ok(A, m, n)) return -4;
  HIPCHK(launch_renorm(prec, m, n, zm(A), (hipStream_t)stream));
  return 0;
}

int mplu_zconvert(int prec_src, int prec_dst, int64_t m, int64_t n, mplu_zmat_t A,
                  mplu_zmat_t B, void *stream) {
  if (!prec_ok(prec_src)) return -1;
  if (!prec_ok(prec_dst)) return -2;
  if (m < 0) return -3;
  if (n < 0) return -4;
  if (!mat_ok(A, m, n)) return -5;
  if (!mat_ok(B, m, n)) return -6;
  HIPCHK(launch_convert(prec_src, prec_dst, m, n, zm(A), zm(B), (hipStream_t)stream));
  return 0;
}

int mplu_zgetrf_wsbytes(int prec, int64_t m, int64_t n, const mplu_opts_t *opts,
                        size_t *bytes) {
  if (!prec_ok(prec)) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!bytes) return -5;
  return getrf_ws(prec, m, n, opts, bytes);
}

}  // extern "C"

namespace {

// the blocked factorisation of mplu_zgetrf; real = true runs the trailing updates with the
// real product (the imaginary planes of A must then be zero and stay so)
int getrf_core(int prec, int64_t m, int64_t n, mplu_zmat_t A, int32_t *d_ipiv,
               int32_t *d_info, const mplu_opts_t *opts, void *d_work, size_t work_bytes,
               void *stream, bool real) {
  if (!prec_ok(prec)) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!mat_ok(A, m, n)) return -4;
  const int64_t mn = m < n ? m : n;
  if (mn > 0 && d_ipiv == nullptr) return -5;
  if (d_info == nullptr) return -6;
  if (opts && (opts->panel < 0 ||
               (opts->flags & ~(MPLU_FLAG_NO_LOOKAHEAD | MPLU_FLAG_EXPIRE_WAITS)) != 0))
    return -7;
  const int method = gemm_method(opts);
  if (method != MPLU_GEMM_4M && method != MPLU_GEMM_3M && method != MPLU_GEMM_SPLIT_F64 &&
      method != MPLU_GEMM_SPLIT_I8 && method != MPLU_GEMM_STRASSEN)
    return -7;
  if (real && method == MPLU_GEMM_STRASSEN) return MPLU_E_UNSUPPORTED;
  if (!split_opts_ok(prec, method, opts)) return MPLU_E_UNSUPPORTED;
  {
    // the panel is held in LDS: widths up to kMaxPanel (a width >= min(m, n) asks for the
    // unblocked factorisation, so it needs min(m, n) <= kMaxPanel)
    const int64_t req = (opts && opts->panel > 0) ? opts->panel : kDefaultPanel;
    if ((req < mn ? req : mn) > kMaxPanel) return MPLU_E_UNSUPPORTED;
  }
  size_t need = 0;
  getrf_ws(prec, m, n, opts, &need);
  if (d_work == nullptr || ((uintptr_t)d_work & 255u)) return -8;
  if (work_bytes < need) return MPLU_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int C = prec;
  int kb = panel_width(opts);
  if (mn > 0 && kb > mn) kb = (int)mn;
  // the panel must fit its grid of co-resident workgroups
  for (int64_t j = 0; j < mn; j += kb) {
    const int jb = (int)((mn - j) < kb ? (mn - j) : kb);
    if (panel_geometry(C, m - j, jb).G == 0) return MPLU_E_UNSUPPORTED;
  }
  HIPCHK(launch_fill_i32(d_info, 0, 1, s));
  if (mn == 0) return 0;
  const ZM a = zm(A);
  const GetrfWS L = getrf_layout(C, m, n, opts);
  char *wb = (char *)d_work;
  void *pws[3] = {wb, wb + L.panel, wb + 2 * L.panel};
  void *split_rest = wb + 3 * L.panel;
  void *split_next = wb + 3 * L.panel + L.split_rest;
  const int S = opts ? opts->n_slices : 0;

  unsigned base[3] = {0u, 0u, 0u};
  const bool expire = opts && (opts->flags & MPLU_FLAG_EXPIRE_WAITS);
  for (int i = 0; i < 3; ++i) HIPCHK(panel_ws_clear(pws[i], expire, s));
  const hipStream_t b = opts ? (hipStream_t)opts->aux_stream : nullptr;
  if (b == nullptr || b == s || (opts->flags & MPLU_FLAG_NO_LOOKAHEAD)) {
    for (int64_t j = 0; j < mn; j += kb) {
      const int jb = (int)((mn - j) < kb ? (mn - j) : kb);
      HIPCHK(launch_panel(C, a, j, m, jb, d_ipiv, d_info, pws[0], &base[0], s, real));
      HIPCHK(launch_laswp(C, a, j, j + jb, n, pws[0], jb, s, real));
      HIPCHK(step_update(C, method, S, a, m, j, jb, j + jb, n, split_rest, s, real));
    }
    return 0;
  }

  // Look-ahead by one panel.  After panel k (columns [j, j+jb)) is factored:
  //   stream `s`:       interchanges, U12 and A22 update of the next panel's columns,
  //                     then panel k+1;
  //   second stream b:  interchanges and U12 of the columns right of the next panel, their
  //                     A22 update, then the interchanges of the columns left of panel k
  //                     (nothing reads those before the end).
  // The next panel's columns are up to date through step k-1 only after the second
  // stream's step k-1 product, which `s` waits for first.  b first waits for everything
  // enqueued on `s` before this call (the event recorded before panel 0), and `s` waits
  // for all of b's work at the end, so the call is one ordered unit of work on `s`.
  LookaheadEvents ev;
  HIPCHK(ev.create());
  HIPCHK(launch_panel(C, a, 0, m, (int)(mn < kb ? mn : kb), d_ipiv, d_info, pws[0], &base[0], s,
                      real));
  int k = 0;
  for (int64_t j = 0; j < mn; j += kb, ++k) {
    const int jb = (int)((mn - j) < kb ? (mn - j) : kb);
    void *pw = pws[k % 3];
    const int64_t nx0 = j + jb;  // next panel's columns [nx0, nx1)
    const int64_t nx1 = nx0 < mn ? nx0 + ((mn - nx0) < kb ? (mn - nx0) : kb) : nx0;
    HIPCHK(hipEventRecord(ev.panel, s));
    if (k > 0) HIPCHK(hipStreamWaitEvent(s, ev.rest, 0));
    HIPCHK(hipStreamWaitEvent(b, ev.panel, 0));
    if (nx1 > nx0) {
      // the next panel's columns: interchanges and U12 in one launch, then the product
      // (with Strassen chosen, this narrow product on the critical path stays plain 3M:
      // the fifteen block sums would only add launches to it)
      HIPCHK(step_trsm(C, a, j, jb, nx0, nx1, s, panel_swap_list(pw, C, jb), real, true));
      HIPCHK(step_gemm(C, method == MPLU_GEMM_STRASSEN ? MPLU_GEMM_3M : method, S, a, m, j, jb,
                       nx0, nx1, split_next, s, real, true));
    }
    // the second stream's product waits until the next panel is about to start, so the
    // panel's workgroups are dispatched before the product fills the device
    HIPCHK(hipEventRecord(ev.chain, s));
    HIPCHK(step_trsm(C, a, j, jb, nx1, n, b, panel_swap_list(pw, C, jb), real));
    HIPCHK(hipStreamWaitEvent(b, ev.chain, 0));
    HIPCHK(step_gemm(C, method, S, a, m, j, jb, nx1, n, split_rest, b, real));
    HIPCHK(hipEventRecord(ev.rest, b));
    // panel k's interchanges on the columns left of it; the workspace holding the list is
    // next written by panel k+3, which the caller's stream starts only after the second
    // stream's step k+1 product
    HIPCHK(launch_laswp(C, a, j, n, n, pw, jb, b, real));
    if (nx1 > nx0)
      HIPCHK(launch_panel(C, a, nx0, m, (int)(nx1 - nx0), d_ipiv, d_info, pws[(k + 1) % 3],
                          &base[(k + 1) % 3], s, real));
  }
  HIPCHK(hipEventRecord(ev.rest, b));
  HIPCHK(hipStreamWaitEvent(s, ev.rest, 0));
  return 0;
}

}  // namespace

extern "C" {

int mplu_zgetrf(int prec, int64_t m, int64_t n, mplu_zmat_t A, int32_t *d_ipiv,
                int32_t *d_info, const mplu_opts_t *opts, void *d_work, size_t work_bytes,
                void *stream) {
  return getrf_core(prec, m, n, A, d_ipiv, d_info, opts, d_work, work_bytes, stream, false);
}

int mplu_zgetrs_wsbytes(int prec, int64_t n, int64_t nrhs, size_t *bytes) {
  if (!prec_ok(prec)) return -1;
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (!bytes) return -4;
  return getrs_ws(prec, n, nrhs, bytes);
}

}  // extern "C"

namespace {

// the substitutions of mplu_zgetrs; real = true: real matrices (C planes; trans 'C' is
// then the transpose)
int getrs_core(int prec, char trans, int64_t n, int64_t nrhs, mplu_zmat_t LU,
               const int32_t *d_ipiv, mplu_zmat_t B, void *d_work, size_t work_bytes,
               void *stream, bool real) {
  if (!prec_ok(prec)) return -1;
  if (trans != 'N' && trans != 'C') return -2;
  if (n < 0) return -3;
  if (nrhs < 0) return -4;
  if (!mat_ok(LU, n, n)) return -5;
  if (n > 0 && d_ipiv == nullptr) return -6;
  if (!mat_ok(B, n, nrhs)) return -7;
  size_t need = 0;
  getrs_ws(prec, n, nrhs, &need);
  if (d_work == nullptr || ((uintptr_t)d_work & 255u)) return -8;
  if (work_bytes < need) return MPLU_E_WORKSPACE;
  if (n == 0 || nrhs == 0) return 0;
  if (n > INT32_MAX) return MPLU_E_UNSUPPORTED;  // 1-based int32 pivot indices
  hipStream_t s = (hipStream_t)stream;
  const int C = prec;
  int32_t *perm = (int32_t *)d_work;
  double *wbuf = (double *)((char *)d_work + align256(sizeof(int32_t) * (size_t)n));
  const ZM w{wbuf, n, n * nrhs};
  const ZM lu = zm(LU), b = zm(B);
  HIPCHK(launch_perm(d_ipiv, n, perm, s));
  if (nrhs <= kSvMaxRhs) {
    int32_t *flags = (int32_t *)((char *)wbuf + align256(sizeof(double) * 2 * C * (size_t)n * (size_t)nrhs));
    if (trans == 'N') {
      HIPCHK(launch_gather_rows(C, perm, n, nrhs, b, w, false, s, real));            // P b
      HIPCHK(launch_trsv(C, true, true, false, lu, w, n, nrhs, flags, s, real));      // L y = P b
      HIPCHK(launch_trsv(C, false, false, false, lu, w, n, nrhs, flags, s, real));    // U x = y
      HIPCHK(launch_gather_rows(C, nullptr, n, nrhs, b, w, true, s, real));
    } else {
      HIPCHK(launch_gather_rows(C, nullptr, n, nrhs, b, w, false, s, real));
      HIPCHK(launch_trsv(C, false, false, true, lu, w, n, nrhs, flags, s, real));     // U^H z = b
      HIPCHK(launch_trsv(C, true, true, true, lu, w, n, nrhs, flags, s, real));       // L^H w = z
      HIPCHK(launch_gather_rows(C, perm, n, nrhs, b, w, true, s, real));              // x = P^T w
    }
    return 0;
  }
  const int NB = kSolveBlock;
  const int gm = real ? 2 : 0;  // block updates: the real product, else 4M
  const int64_t nblk = (n + NB - 1) / NB;
  if (trans == 'N') {
    HIPCHK(launch_gather_rows(C, perm, n, nrhs, b, w, false, s, real));
    for (int64_t bi = 0; bi < nblk; ++bi) {  // L y = P b
      const int64_t i0 = bi * NB;
      const int nb = (int)((n - i0) < NB ? (n - i0) : NB);
      HIPCHK(launch_trsm(C, true, true, false, lu, i0, nb, w, i0, 0, nrhs, s, nullptr, 0, real));
      if (i0 + nb < n)
        HIPCHK(launch_gemm(C, gm, 'N', 'N', n - i0 - nb, nrhs, nb, -1, lu, i0 + nb, i0, w, i0, 0,
                           1, w, i0 + nb, 0, s));
    }
    for (int64_t bi = nblk - 1; bi >= 0; --bi) {  // U x = y
      const int64_t i0 = bi * NB;
      const int nb = (int)((n - i0) < NB ? (n - i0) : NB);
      HIPCHK(launch_trsm(C, false, false, false, lu, i0, nb, w, i0, 0, nrhs, s, nullptr, 0, real));
      if (i0 > 0)
        HIPCHK(launch_gemm(C, gm, 'N', 'N', i0, nrhs, nb, -1, lu, 0, i0, w, i0, 0, 1, w, 0, 0, s));
    }
    // W holds x in natural order: identity copy back
    HIPCHK(launch_gather_rows(C, nullptr, n, nrhs, b, w, true, s, real));
  } else {
    HIPCHK(launch_gather_rows(C, nullptr, n, nrhs, b, w, false, s, real));
    for (int64_t bi = 0; bi < nblk; ++bi) {  // U^H z = b
      const int64_t i0 = bi * NB;
      const int nb = (int)((n - i0) < NB ? (n - i0) : NB);
      HIPCHK(launch_trsm(C, false, false, true, lu, i0, nb, w, i0, 0, nrhs, s, nullptr, 0, real));
      if (i0 + nb < n)
        HIPCHK(launch_gemm(C, gm, 'C', 'N', n - i0 - nb, nrhs, nb, -1, lu, i0, i0 + nb, w, i0, 0,
                           1, w, i0 + nb, 0, s));
    }
    for (int64_t bi = nblk - 1; bi >= 0; --bi) {  // L^H w = z
      const int64_t i0 = bi * NB;
      const int nb = (int)((n - i0) < NB ? (n - i0) : NB);
      HIPCHK(launch_trsm(C, true, true, true, lu, i0, nb, w, i0, 0, nrhs, s, nullptr, 0, real));
      if (i0 > 0)
        HIPCHK(launch_gemm(C, gm, 'C', 'N', i0, nrhs, nb, -1, lu, i0, 0, w, i0, 0, 1, w, 0, 0, s));
    }
    HIPCHK(launch_gather_rows(C, perm, n, nrhs, b, w, true, s, real));  // x = P^T w
  }
  return 0;
}

}  // namespace

extern "C" {

int mplu_zgetrs(int prec, char trans, int64_t n, int64_t nrhs, mplu_zmat_t LU,
                const int32_t *d_ipiv, mplu_zmat_t B, void *d_work, size_t work_bytes,
                void *stream) {
  return getrs_core(prec, trans, n, nrhs, LU, d_ipiv, B, d_work, work_bytes, stream, false);
}

int mplu_zgesv_wsbytes(int prec, int64_t n, int64_t nrhs, const mplu_opts_t *opts,
                       size_t *bytes) {
  if (!prec_ok(prec)) return -1;
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (!bytes) return -5;
  size_t a = 0, b = 0;
  getrf_ws(prec, n, n, opts, &a);
  getrs_ws(prec, n, nrhs, &b);
  *bytes = a > b ? a : b;
  return 0;
}

int mplu_zgesv(int prec, int64_t n, int64_t nrhs, mplu_zmat_t A, int32_t *d_ipiv,
               mplu_zmat_t B, int32_t *d_info, const mplu_opts_t *opts, void *d_work,
               size_t work_bytes, void *stream) {
  if (!prec_ok(prec)) return -1;
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (!mat_ok(A, n, n)) return -4;
  if (n > 0 && d_ipiv == nullptr) return -5;
  if (!mat_ok(B, n, nrhs)) return -6;
  if (d_info == nullptr) return -7;
  size_t need = 0;
  mplu_zgesv_wsbytes(prec, n, nrhs, opts, &need);
  if (d_work == nullptr || ((uintptr_t)d_work & 255u)) return -9;
  if (work_bytes < need) return MPLU_E_WORKSPACE;
  int rc = mplu_zgetrf(prec, n, n, A, d_ipiv, d_info, opts, d_work, work_bytes, stream);
  if (rc == -7) return -8;  // the options (the only argument not checked above)
  if (rc != 0) return rc;
  return mplu_zgetrs(prec, 'N', n, nrhs, A, d_ipiv, B, d_work, work_bytes, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ no-allocation gesv
// mplu_zgesv_noalloc takes its workspace from this array instead of the caller.  Each
// device holds its own copy at its own address, looked up once per device; host code
// only ever hands kernels that address, never the array's name.
namespace {

constexpr size_t kScratchBytes = (size_t)MPLU_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::atomic<void *> g_scratch_ptr[kMaxDevices];

// device address of the current device's scratch (nullptr if the lookup failed)
void *scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (p) return p;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
  if (p) return p;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
  g_scratch_ptr[dev].store(p, std::memory_order_release);
  return p;
}

}  // namespace

extern "C" {

int mplu_zgesv_noalloc(int prec, int64_t n, int64_t nrhs, mplu_zmat_t A, int32_t *d_ipiv,
                       mplu_zmat_t B, int32_t *d_info, const mplu_opts_t *opts,
                       void *stream) {
  if (!prec_ok(prec)) return -1;
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (!mat_ok(A, n, n)) return -4;
  if (n > 0 && d_ipiv == nullptr) return -5;
  if (!mat_ok(B, n, nrhs)) return -6;
  if (d_info == nullptr) return -7;
  // every step in order on `stream`: the look-ahead's second stream and its events are
  // left out, so nothing is created here
  mplu_opts_t o = opts ? *opts : mplu_opts_t{0, MPLU_GEMM_3M, 0, 0, 0, nullptr};
  if (o.panel < 0 || (o.flags & ~(MPLU_FLAG_NO_LOOKAHEAD | MPLU_FLAG_EXPIRE_WAITS)) != 0)
    return -8;
  o.flags |= MPLU_FLAG_NO_LOOKAHEAD;
  o.aux_stream = nullptr;
  size_t need = 0;
  if (mplu_zgesv_wsbytes(prec, n, nrhs, &o, &need) != 0) return -8;
  if (need > kScratchBytes) return MPLU_E_SCRATCH;
  void *ws = scratch_ptr();
  if (ws == nullptr) return MPLU_E_HIP;
  int rc = getrf_core(prec, n, n, A, d_ipiv, d_info, &o, ws, kScratchBytes, stream, false);
  if (rc == -7) return -8;
  if (rc != 0) return rc;
  return getrs_core(prec, 'N', n, nrhs, A, d_ipiv, B, ws, kScratchBytes, stream, false);
}

int mplu_zgemm_wsbytes(int prec, int64_t m, int64_t n, int64_t k, int method,
                       const mplu_opts_t *opts, size_t *bytes) {
  if (!prec_ok(prec)) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (k < 0) return -4;
  if (method < 0 || method > MPLU_GEMM_STRASSEN) return -5;
  if (!bytes) return -7;
  *bytes = is_split(method) ? split_ws_bytes(prec, method == MPLU_GEMM_SPLIT_I8, m, n, k,
                                             opts ? opts->n_slices : 0)
           : method == MPLU_GEMM_STRASSEN ? strassen_ws(prec, m, n, k)
                                          : 0;
  return 0;
}

int mplu_zgemm(int prec, char opA, char opB, int64_t m, int64_t n, int64_t k, int alpha_sign,
               mplu_zmat_t A, mplu_zmat_t B, int beta, mplu_zmat_t Cm, int method,
               const mplu_opts_t *opts, void *d_work, size_t work_bytes, void *stream) {
  if (!prec_ok(prec)) return -1;
  if (opA != 'N' && opA != 'T' && opA != 'C') return -2;
  if (opB != 'N' && opB != 'T' && opB != 'C') return -3;
  if (m < 0) return -4;
  if (n < 0) return -5;
  if (k < 0) return -6;
  if (alpha_sign != 1 && alpha_sign != -1) return -7;
  if (!mat_ok(A, opA == 'N' ? m : k, opA == 'N' ? k : m)) return -8;
  if (!mat_ok(B, opB == 'N' ? k : n, opB == 'N' ? n : k)) return -9;
  if (beta != 0 && beta != 1) return -10;
  if (!mat_ok(Cm, m, n)) return -11;
  if (method < 0 || method > MPLU_GEMM_STRASSEN) return -12;
  if (opts && opts->flags != 0) return -13;
  if (method == MPLU_GEMM_STRASSEN) {
    if (opA != 'N' || opB != 'N') return MPLU_E_UNSUPPORTED;
    size_t need = 0;
    mplu_zgemm_wsbytes(prec, m, n, k, method, opts, &need);
    if (m > 0 && n > 0 && (d_work == nullptr || ((uintptr_t)d_work & 255u))) return -14;
    if (work_bytes < need) return MPLU_E_WORKSPACE;
    HIPCHK(strassen_zgemm(prec, m, n, k, alpha_sign, zm(A), zm(B), beta, zm(Cm), d_work,
                          (hipStream_t)stream));
    return 0;
  }
  if (is_split(method)) {
    if (!split_opts_ok(prec, method, opts)) return MPLU_E_UNSUPPORTED;
    size_t need = 0;
    mplu_zgemm_wsbytes(prec, m, n, k, method, opts, &need);
    if (m > 0 && n > 0 && (d_work == nullptr || ((uintptr_t)d_work & 255u))) return -14;
    if (work_bytes < need) return MPLU_E_WORKSPACE;
    HIPCHK(launch_gemm_split(prec, method == MPLU_GEMM_SPLIT_I8, opts ? opts->n_slices : 0, opA,
                             opB, m, n, k, alpha_sign, zm(A), 0, 0, zm(B), 0, 0, beta, zm(Cm), 0,
                             0, d_work, (hipStream_t)stream));
    return 0;
  }
  HIPCHK(launch_gemm(prec, method == MPLU_GEMM_3M ? 1 : 0, opA, opB, m, n, k, alpha_sign, zm(A),
                     0, 0, zm(B), 0, 0, beta, zm(Cm), 0, 0, (hipStream_t)stream));
  return 0;
}

// ------------------------------------------------------------------ real matrices
// The Im = 0 case with the same kernels in their real variants (C planes per value): the
// panel, interchanges, triangular solves and substitutions on real values, the real
// product for the trailing updates and block updates.

static inline bool dmat_ok(const mplu_dmat_t &A, int64_t rows, int64_t cols) {
  return mat_ok(mplu_zmat_t{A.planes, A.ld, A.plane_stride}, rows, cols);
}

static inline ZM dm(const mplu_dmat_t &A) { return ZM{A.planes, A.ld, A.plane_stride}; }

// the descriptor as the internal routines take it (only its first C planes are touched)
static inline mplu_zmat_t as_z(const mplu_dmat_t &A) {
  return mplu_zmat_t{A.planes, A.ld, A.plane_stride};
}

int mplu_dgetrf_wsbytes(int prec, int64_t m, int64_t n, const mplu_opts_t *opts,
                        size_t *bytes) {
  if (!prec_ok(prec)) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!bytes) return -5;
  return getrf_ws(prec, m, n, opts, bytes);
}

int mplu_dgetrf(int prec, int64_t m, int64_t n, mplu_dmat_t A, int32_t *d_ipiv,
                int32_t *d_info, const mplu_opts_t *opts, void *d_work, size_t work_bytes,
                void *stream) {
  if (!prec_ok(prec)) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!dmat_ok(A, m, n)) return -4;
  return getrf_core(prec, m, n, as_z(A), d_ipiv, d_info, opts, d_work, work_bytes, stream,
                    true);
}

int mplu_dgetrs_wsbytes(int prec, int64_t n, int64_t nrhs, size_t *bytes) {
  if (!prec_ok(prec)) return -1;
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (!bytes) return -4;
  return getrs_ws(prec, n, nrhs, bytes);
}

int mplu_dgetrs(int prec, char trans, int64_t n, int64_t nrhs, mplu_dmat_t LU,
                const int32_t *d_ipiv, mplu_dmat_t B, void *d_work, size_t work_bytes,
                void *stream) {
  if (!prec_ok(prec)) return -1;
  if (trans != 'N' && trans != 'T') return -2;
  // A^T of a real matrix is what the complex routine calls A^H
  return getrs_core(prec, trans == 'N' ? 'N' : 'C', n, nrhs, as_z(LU), d_ipiv, as_z(B),
                    d_work, work_bytes, stream, true);
}

int mplu_dgesv_wsbytes(int prec, int64_t n, int64_t nrhs, const mplu_opts_t *opts,
                       size_t *bytes) {
  if (!prec_ok(prec)) return -1;
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (!bytes) return -5;
  size_t a = 0, b = 0;
  getrf_ws(prec, n, n, opts, &a);
  getrs_ws(prec, n, nrhs, &b);
  *bytes = a > b ? a : b;
  return 0;
}

int mplu_dgesv(int prec, int64_t n, int64_t nrhs, mplu_dmat_t A, int32_t *d_ipiv,
               mplu_dmat_t B, int32_t *d_info, const mplu_opts_t *opts, void *d_work,
               size_t work_bytes, void *stream) {
  if (!prec_ok(prec)) return -1;
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (!dmat_ok(A, n, n)) return -4;
  if (n > 0 && d_ipiv == nullptr) return -5;
  if (!dmat_ok(B, n, nrhs)) return -6;
  if (d_info == nullptr) return -7;
  size_t need = 0;
  mplu_dgesv_wsbytes(prec, n, nrhs, opts, &need);
  if (d_work == nullptr || ((uintptr_t)d_work & 255u)) return -9;
  if (work_bytes < need) return MPLU_E_WORKSPACE;
  int rc = getrf_core(prec, n, n, as_z(A), d_ipiv, d_info, opts, d_work, work_bytes, stream,
                      true);
  if (rc == -7) return -8;  // the options (the only argument not checked above)
  if (rc != 0) return rc;
  return getrs_core(prec, 'N', n, nrhs, as_z(A), d_ipiv, as_z(B), d_work, work_bytes, stream,
                    true);
}

int mplu_dgemm(int prec, char opA, char opB, int64_t m, int64_t n, int64_t k, int alpha_sign,
               mplu_dmat_t A, mplu_dmat_t B, int beta, mplu_dmat_t Cm, void *stream) {
  if (!prec_ok(prec)) return -1;
  if (opA != 'N' && opA != 'T') return -2;
  if (opB != 'N' && opB != 'T') return -3;
  if (m < 0) return -4;
  if (n < 0) return -5;
  if (k < 0) return -6;
  if (alpha_sign != 1 && alpha_sign != -1) return -7;
  if (!dmat_ok(A, opA == 'N' ? m : k, opA == 'N' ? k : m)) return -8;
  if (!dmat_ok(B, opB == 'N' ? k : n, opB == 'N' ? n : k)) return -9;
  if (beta != 0 && beta != 1) return -10;
  if (!dmat_ok(Cm, m, n)) return -11;
  HIPCHK(launch_gemm(prec, 2, opA, opB, m, n, k, alpha_sign, dm(A), 0, 0, dm(B), 0, 0, beta,
                     dm(Cm), 0, 0, (hipStream_t)stream));
  return 0;
}

}  // extern "C"
