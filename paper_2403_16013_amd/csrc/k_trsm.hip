// k_trsm.hip -- solve op(T) X = X for one nb x nb triangular block T (nb <= 128),
// in place, many right-hand-side columns at once.
//
// Used for the block row of U in the blocked LU (U12 := L11^-1 A12, Kouya Sec. 3) and for
// the diagonal blocks of the forward / backward substitutions (Sec. 4).  Each workgroup
// owns a strip of columns of X held in LDS, stages the triangle in LDS and sweeps the nb
// rows in order.  Blocks whose triangle does not fit are split in halves around a 4M
// product.  Element operations use the 4M complex product with one rounding per part
// (Eq. 4m).
#include "common.hpp"

#pragma clang fp contract(off)

namespace mplu {

struct TrsmArgs {
  ZM T;
  int64_t t0;
  int nb;
  ZM X;
  int64_t x0, c0, ncols;
  int nbc;  // columns per workgroup
};

// op(T)[r][i]
template <int C, bool CONJ>
__device__ __forceinline__ void ld_opT(const TrsmArgs &a, int r, int i, double (&re)[C],
                                       double (&im)[C]) {
  if (CONJ) {
    ld_z<C>(a.T, a.t0 + i, a.t0 + r, re, im);
#pragma unroll
    for (int c = 0; c < C; ++c) im[c] = -im[c];
  } else {
    ld_z<C>(a.T, a.t0 + r, a.t0 + i, re, im);
  }
}

// LOWER: op(T) is lower triangular (forward sweep); UNIT: unit diagonal.
// The strict triangle of op(T) is staged once in LDS, packed by columns in component
// planes (column i holds rows i+1..nb-1 when LOWER, rows 0..i-1 otherwise), so the sweep
// reads it at LDS latency; the diagonal is kept as reciprocals.
template <int C, bool LOWER, bool UNIT, bool CONJ>
__global__ __launch_bounds__(256) void k_trsm(TrsmArgs a) {
  extern __shared__ double smem[];
  constexpr int Q = 2 * C;
  const int nb = a.nb, NBC = a.nbc, t = threadIdx.x;
  const int ntri = nb * (nb - 1) / 2;
  const int64_t cb = a.c0 + (int64_t)blockIdx.x * NBC;
  const int64_t left = a.c0 + a.ncols - cb;
  const int ncl = (int)(left < NBC ? left : NBC);
  double *sX = smem;                          // [nb][Q][NBC]
  double *sR = sX + (size_t)nb * Q * NBC;     // [nb][Q] reciprocals of the diagonal
  double *sT = sR + (size_t)nb * Q;           // [Q][ntri] packed strict triangle

  auto col_off = [&](int i) { return LOWER ? i * (nb - 1) - i * (i - 1) / 2 : i * (i - 1) / 2; };

  for (int e = t; e < nb * ncl * Q; e += 256) {
    const int r = e % nb, rest = e / nb, cc = rest % ncl, q = rest / ncl;
    sX[((size_t)r * Q + q) * NBC + cc] = a.X.p[(int64_t)q * a.X.ps + (cb + cc) * a.X.ld + a.x0 + r];
  }
  // strict triangle: enumerate (column i, row r) pairs column by column
  for (int e = t; e < ntri; e += 256) {
    int i, r;
    if (LOWER) {  // column i has nb-1-i entries
      i = 0;
      int acc = 0;
      while (acc + (nb - 1 - i) <= e) { acc += nb - 1 - i; ++i; }
      r = i + 1 + (e - acc);
    } else {      // column i has i entries
      i = 1;
      int acc = 0;
      while (acc + i <= e) { acc += i; ++i; }
      r = e - acc;
    }
    double tr[C], ti[C];
    ld_opT<C, CONJ>(a, r, i, tr, ti);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      sT[(size_t)c * ntri + e] = tr[c];
      sT[(size_t)(C + c) * ntri + e] = ti[c];
    }
  }
  if (!UNIT) {
    for (int i = t; i < nb; i += 256) {
      double dr[C], di[C], rr[C], ri[C];
      ld_opT<C, CONJ>(a, i, i, dr, di);
      mp::zrecip<C>(dr, di, rr, ri);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        sR[i * Q + c] = rr[c];
        sR[i * Q + C + c] = ri[c];
      }
    }
  }
  __syncthreads();

  for (int s = 0; s < nb; ++s) {
    const int i = LOWER ? s : nb - 1 - s;
    if (!UNIT) {
      for (int cc = t; cc < ncl; cc += 256) {
        double xr[C], xi[C], rr[C], ri[C], orr[C], oi[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          xr[c] = sX[((size_t)i * Q + c) * NBC + cc];
          xi[c] = sX[((size_t)i * Q + C + c) * NBC + cc];
          rr[c] = sR[i * Q + c];
          ri[c] = sR[i * Q + C + c];
        }
        mp::zmul<C>(xr, xi, rr, ri, orr, oi);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          sX[((size_t)i * Q + c) * NBC + cc] = orr[c];
          sX[((size_t)i * Q + C + c) * NBC + cc] = oi[c];
        }
      }
      __syncthreads();
    }
    const int rlo = LOWER ? i + 1 : 0;
    const int rcnt = LOWER ? nb - i - 1 : i;
    const int off = col_off(i);
    for (int e = t; e < rcnt * ncl; e += 256) {
      const int r = rlo + e / ncl, cc = e % ncl;
      double tr[C], ti[C], xr[C], xi[C], yr[C], yi[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        tr[c] = sT[(size_t)c * ntri + off + (r - rlo)];
        ti[c] = sT[(size_t)(C + c) * ntri + off + (r - rlo)];
        xr[c] = sX[((size_t)r * Q + c) * NBC + cc];
        xi[c] = sX[((size_t)r * Q + C + c) * NBC + cc];
        yr[c] = sX[((size_t)i * Q + c) * NBC + cc];
        yi[c] = sX[((size_t)i * Q + C + c) * NBC + cc];
      }
      mp::zfms<C>(xr, xi, tr, ti, yr, yi, xr, xi);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        sX[((size_t)r * Q + c) * NBC + cc] = xr[c];
        sX[((size_t)r * Q + C + c) * NBC + cc] = xi[c];
      }
    }
    __syncthreads();
  }

  for (int e = t; e < nb * ncl * Q; e += 256) {
    const int r = e % nb, rest = e / nb, cc = rest % ncl, q = rest / ncl;
    a.X.p[(int64_t)q * a.X.ps + (cb + cc) * a.X.ld + a.x0 + r] = sX[((size_t)r * Q + q) * NBC + cc];
  }
}

template <int C, bool LOWER, bool UNIT, bool CONJ>
static hipError_t go(const TrsmArgs &a, hipStream_t s) {
  constexpr int Q = 2 * C;
  const size_t lds = sizeof(double) * ((size_t)a.nb * Q * a.nbc + (size_t)a.nb * Q +
                                        (size_t)Q * (a.nb * (a.nb - 1) / 2));
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k_trsm<C, LOWER, UNIT, CONJ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t blocks = (a.ncols + a.nbc - 1) / a.nbc;
  hipLaunchKernelGGL((k_trsm<C, LOWER, UNIT, CONJ>), dim3((unsigned)blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int C>
static hipError_t dispatch(bool lower, bool unit, bool conj, const TrsmArgs &a, hipStream_t s) {
  // op(T) is lower when T is lower and not transposed, or T upper and transposed
  const bool opl = lower != conj;
  if (opl) {
    if (unit) return conj ? go<C, true, true, true>(a, s) : go<C, true, true, false>(a, s);
    return conj ? go<C, true, false, true>(a, s) : go<C, true, false, false>(a, s);
  }
  if (unit) return conj ? go<C, false, true, true>(a, s) : go<C, false, true, false>(a, s);
  return conj ? go<C, false, false, true>(a, s) : go<C, false, false, false>(a, s);
}

static inline size_t tri_fixed(int C, int nb) {
  return sizeof(double) * 2 * C * ((size_t)nb + (size_t)nb * (nb - 1) / 2);
}

hipError_t launch_trsm(int C, bool lower, bool unit, bool conj, ZM Tm, int64_t t0, int nb,
                       ZM Xm, int64_t x0, int64_t c0, int64_t ncols, hipStream_t s) {
  if (nb <= 0 || ncols <= 0) return hipSuccess;
  if (tri_fixed(C, nb) + sizeof(double) * 2 * C * nb > 128 * 1024) {
    // the packed triangle does not fit: split op(T) into halves,
    //   lower op:  X1 = T11^-1 X1;  X2 -= T21 X1;  X2 = T22^-1 X2
    //   upper op:  X2 = T22^-1 X2;  X1 -= T12 X2;  X1 = T11^-1 X1
    const int h = nb / 2, r = nb - h;
    const bool opl = lower != conj;
    const char opA = conj ? 'C' : 'N';
    hipError_t e;
    if (opl) {
      if ((e = launch_trsm(C, lower, unit, conj, Tm, t0, h, Xm, x0, c0, ncols, s)) != hipSuccess) return e;
      // T21 = op(T)[h:, :h]: stored at (t0+h, t0) untransposed, else (t0, t0+h) transposed
      if ((e = launch_gemm(C, 0, opA, 'N', r, ncols, h, -1, Tm, conj ? t0 : t0 + h,
                           conj ? t0 + h : t0, Xm, x0, c0, 1, Xm, x0 + h, c0, s)) != hipSuccess)
        return e;
      return launch_trsm(C, lower, unit, conj, Tm, t0 + h, r, Xm, x0 + h, c0, ncols, s);
    }
    if ((e = launch_trsm(C, lower, unit, conj, Tm, t0 + h, r, Xm, x0 + h, c0, ncols, s)) != hipSuccess) return e;
    // T12 = op(T)[:h, h:]: stored at (t0, t0+h) untransposed, else (t0+h, t0) transposed
    if ((e = launch_gemm(C, 0, opA, 'N', h, ncols, r, -1, Tm, conj ? t0 + h : t0,
                         conj ? t0 : t0 + h, Xm, x0 + h, c0, 1, Xm, x0, c0, s)) != hipSuccess)
      return e;
    return launch_trsm(C, lower, unit, conj, Tm, t0, h, Xm, x0, c0, ncols, s);
  }
  TrsmArgs a;
  a.T = Tm;
  a.t0 = t0;
  a.nb = nb;
  a.X = Xm;
  a.x0 = x0;
  a.c0 = c0;
  a.ncols = ncols;
  // columns per workgroup: the packed triangle and the diagonal take their share of the
  // LDS, the column strip the rest (at most 16 columns)
  const size_t fixed = tri_fixed(C, nb);
  int nbc = 16;
  while (nbc > 1 && fixed + sizeof(double) * (size_t)nb * 2 * C * nbc > 160 * 1024) nbc >>= 1;
  a.nbc = nbc;
  switch (C) {
    case 2: return dispatch<2>(lower, unit, conj, a, s);
    case 3: return dispatch<3>(lower, unit, conj, a, s);
    case 4: return dispatch<4>(lower, unit, conj, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mplu
