// common.hpp -- matrix descriptors, plane access and launcher declarations shared by the
// HIP kernels of the library.
//
// Storage (Kouya Sec. 2.2, Fig. 1): real and imaginary parts are kept apart; each part is
// C binary64 component planes.  Plane q = ri*C + c sits at p + q*ps; within a plane the
// matrix is column-major with leading dimension ld.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "mp.hpp"

#pragma clang fp contract(off)

namespace mplu {

struct ZM {
  double *p;
  int64_t ld;
  int64_t ps;
};

template <int C>
__device__ __forceinline__ void ld_z(const ZM &A, int64_t i, int64_t j, double (&re)[C],
                                     double (&im)[C]) {
  const double *b = A.p + j * A.ld + i;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    re[c] = b[(int64_t)c * A.ps];
    im[c] = b[(int64_t)(C + c) * A.ps];
  }
}

template <int C>
__device__ __forceinline__ void st_z(const ZM &A, int64_t i, int64_t j, const double (&re)[C],
                                     const double (&im)[C]) {
  double *b = A.p + j * A.ld + i;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    b[(int64_t)c * A.ps] = re[c];
    b[(int64_t)(C + c) * A.ps] = im[c];
  }
}

// the real planes only (a real matrix, or the real part of a complex one)
template <int C>
__device__ __forceinline__ void ld_re(const ZM &A, int64_t i, int64_t j, double (&re)[C]) {
  const double *b = A.p + j * A.ld + i;
#pragma unroll
  for (int c = 0; c < C; ++c) re[c] = b[(int64_t)c * A.ps];
}

template <int C>
__device__ __forceinline__ void st_re(const ZM &A, int64_t i, int64_t j, const double (&re)[C]) {
  double *b = A.p + j * A.ld + i;
#pragma unroll
  for (int c = 0; c < C; ++c) b[(int64_t)c * A.ps] = re[c];
}

// Output tile of this workgroup in a 1-D grid of gm x gn tiles.  Workgroups are
// dispatched round-robin over the 8 XCDs; the remap gives each XCD a contiguous range of
// the tile order, and that order walks 8 tile rows down before moving one tile column
// right, so the workgroups an XCD runs together share their rows and columns of the
// operands in its L2.
__device__ __forceinline__ void xcd_tile(int64_t gm, int64_t gn, int64_t &tm, int64_t &tn) {
  constexpr int64_t NX = 8, GR = 8;
  const int64_t total = gm * gn, L = blockIdx.x;
  const int64_t full = total / NX * NX;
  const int64_t id = L < full ? (L % NX) * (total / NX) + L / NX : L;
  const int64_t gsz_all = GR * gn;
  const int64_t grp = id / gsz_all, first = grp * GR;
  const int64_t gsz = (gm - first) < GR ? gm - first : GR;
  const int64_t in = id - grp * gsz_all;
  tm = first + in % gsz;
  tn = in / gsz;
}

// Raise a kernel's dynamic-LDS limit once per device (thread-safe; a failed attempt is
// retried on the next launch).  One static instance per kernel.
struct LdsAttr {
  std::atomic<int> done[64];
  hipError_t ensure(const void *kernel, int bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (done[dev].load(std::memory_order_acquire)) return hipSuccess;
    const hipError_t e =
        hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) done[dev].store(1, std::memory_order_release);
    return e;
  }
};

// ------------------------------------------------------------------ launcher interface
// Every launcher validates nothing (the C ABI does) and returns the launch status.

hipError_t launch_renorm(int C, int64_t m, int64_t n, ZM A, hipStream_t s);
hipError_t launch_convert(int Cs, int Cd, int64_t m, int64_t n, ZM A, ZM B, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s);
// O := sa A + sb B (complex, m x n, sa and sb in {-1, 0, 1}); O may alias A or B
hipError_t launch_zaxpby(int C, int64_t m, int64_t n, int sa, ZM A, int sb, ZM B, ZM O,
                         hipStream_t s);

struct PanelGeom {
  int G;  // workgroups
  int R;  // rows per workgroup
  size_t lds;
};
// choose the panel grid for mp rows and kb columns; G == 0 if it cannot fit
PanelGeom panel_geometry(int C, int64_t mp, int kb);
size_t panel_ws_bytes(int C, int kb);

// clear the barrier words of a panel workspace (once per factorisation, before its
// first panel); expire = true marks its bounded waits as expired (a test of the
// time-out path, forced from the host)
hipError_t panel_ws_clear(void *ws, bool expire, hipStream_t s);
// factor rows [j, m) x columns [j, j+kb) in place; writes ipiv[j..j+kb), info, and the
// swap list for the other columns into the workspace.  *base: barrier arrivals already
// counted on this workspace since it was cleared; advanced past this panel's.
// real = true: A's first C planes hold a real matrix and only those are read or written
// (pivot |a|, real reciprocal)
hipError_t launch_panel(int C, ZM A, int64_t j, int64_t m, int kb, int32_t *ipiv,
                        int32_t *info, void *ws, unsigned *base, hipStream_t s,
                        bool real = false);
// apply the swap list left by launch_panel to columns [0, c0) and [c1, n) (real: C planes)
hipError_t launch_laswp(int C, ZM A, int64_t c0, int64_t c1, int64_t n, const void *ws,
                        int kb, hipStream_t s, bool real = false);

// the interchange list a panel leaves in its workspace (see launch_panel), and the
// interchanges applied to columns [c0, c0+ncols) of A
const int32_t *panel_swap_list(const void *ws, int C, int kb);
hipError_t launch_laswp_list(int C, ZM A, int64_t c0, int64_t ncols, const int32_t *swl,
                             int swstride, hipStream_t s, bool real = false);

// op(T) X = X for an nb x nb triangle T of matrix Tm at (t0, t0), X = rows [x0, x0+nb) x
// cols [c0, c0+ncols) of Xm.  lower: T stored lower; unit: unit diagonal; conj: op = ^H.
// swl (optional): interchange list (as left by a panel of width swstride / 2) applied to
// those columns of Xm first.
// real: real matrices (C planes; conj then means transpose)
// urgent: the solve is on the factorisation's critical path (the next panel's columns);
// its waves raise their issue priority over work of the other stream sharing their CUs
hipError_t launch_trsm(int C, bool lower, bool unit, bool conj, ZM Tm, int64_t t0, int nb,
                       ZM Xm, int64_t x0, int64_t c0, int64_t ncols, hipStream_t s,
                       const int32_t *swl = nullptr, int swstride = 0, bool real = false,
                       bool urgent = false);

// Cm := beta Cm + alpha op(A) op(B);  method 0 = 4M, 1 = 3M, 2 = real (only the real
// planes of A, B and Cm are read, only those of Cm written; 'C' acts as 'T')
// urgent: as for launch_trsm
hipError_t launch_gemm(int C, int method, char opA, char opB, int64_t m, int64_t n, int64_t k,
                       int alpha_sign, ZM A, int64_t ai, int64_t aj, ZM B, int64_t bi,
                       int64_t bj, int beta, ZM Cm, int64_t ci, int64_t cj, hipStream_t s,
                       bool urgent = false);

// split products (Ozaki scheme) for the 3M form: digits on INT8 (i8) or FP64 MFMA; S = 0
// selects the default slice count
int split_slices(int C, bool i8);
bool split_supported(int C, bool i8, int S);
size_t split_ws_bytes(int C, bool i8, int64_t m, int64_t n, int64_t K, int S);
// (real: real operands and result, C planes; one real product instead of three)
hipError_t launch_gemm_split(int C, bool i8, int S, char opA, char opB, int64_t m, int64_t n,
                             int64_t k, int alpha, ZM A, int64_t ai, int64_t aj, ZM B,
                             int64_t bi, int64_t bj, int beta, ZM Cm, int64_t ci, int64_t cj,
                             void *ws, hipStream_t s, bool real = false);

// op(T) X = X for the whole n x n triangle of Tm and nrhs columns of Xm in one launch;
// flags: trsv_flag_words(n, nrhs) int32 of workspace (cleared by the launcher)
int64_t trsv_flag_words(int64_t n, int64_t nrhs);
hipError_t launch_trsv(int C, bool lower, bool unit, bool conj, ZM Tm, ZM Xm, int64_t n,
                       int64_t nrhs, int32_t *flags, hipStream_t s, bool real = false);

// getrs helpers: perm from ipiv (n entries), then gather / scatter rows of B
hipError_t launch_perm(const int32_t *ipiv, int64_t n, int32_t *perm, hipStream_t s);
hipError_t launch_gather_rows(int C, const int32_t *perm, int64_t n, int64_t nrhs, ZM B, ZM W,
                              bool scatter, hipStream_t s, bool real = false);

}  // namespace mplu
