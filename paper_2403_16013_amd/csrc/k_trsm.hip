// k_trsm.hip -- solve op(T) X = X for one nb x nb triangular block T (nb <= 128),
// in place, many right-hand-side columns at once.
//
// Used for the block row of U in the blocked LU (U12 := L11^-1 A12, Kouya Sec. 3) and for
// the diagonal blocks of the forward / backward substitutions (Sec. 4).  Each workgroup
// owns a strip of columns of X held in LDS and sweeps the nb rows in order; the entries
// of T are read from global memory (the block is small and stays in L2).  Element
// operations use the 4M complex product with one rounding per part (Eq. 4m).
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

// LOWER: op(T) is lower triangular (forward sweep); UNIT: unit diagonal
template <int C, bool LOWER, bool UNIT, bool CONJ>
__global__ __launch_bounds__(256) void k_trsm(TrsmArgs a) {
  extern __shared__ double smem[];
  constexpr int Q = 2 * C;
  const int nb = a.nb, NBC = a.nbc, t = threadIdx.x;
  const int64_t cb = a.c0 + (int64_t)blockIdx.x * NBC;
  const int64_t left = a.c0 + a.ncols - cb;
  const int ncl = (int)(left < NBC ? left : NBC);
  double *sX = smem;                          // [nb][Q][NBC]
  double *sR = sX + (size_t)nb * Q * NBC;     // [nb][Q] reciprocals of the diagonal

  for (int e = t; e < nb * ncl * Q; e += 256) {
    const int r = e % nb, rest = e / nb, cc = rest % ncl, q = rest / ncl;
    sX[((size_t)r * Q + q) * NBC + cc] = a.X.p[(int64_t)q * a.X.ps + (cb + cc) * a.X.ld + a.x0 + r];
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
    // rows still to be updated by x_i
    const int rlo = LOWER ? i + 1 : 0;
    const int rcnt = LOWER ? nb - i - 1 : i;
    for (int e = t; e < rcnt * ncl; e += 256) {
      const int r = rlo + e / ncl, cc = e % ncl;
      double tr[C], ti[C], xr[C], xi[C], yr[C], yi[C];
      ld_opT<C, CONJ>(a, r, i, tr, ti);
#pragma unroll
      for (int c = 0; c < C; ++c) {
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
  const size_t lds = sizeof(double) * ((size_t)a.nb * Q * a.nbc + (size_t)a.nb * Q);
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

hipError_t launch_trsm(int C, bool lower, bool unit, bool conj, ZM Tm, int64_t t0, int nb,
                       ZM Xm, int64_t x0, int64_t c0, int64_t ncols, hipStream_t s) {
  if (nb <= 0 || ncols <= 0) return hipSuccess;
  if (nb > 128) return hipErrorInvalidValue;
  TrsmArgs a;
  a.T = Tm;
  a.t0 = t0;
  a.nb = nb;
  a.X = Xm;
  a.x0 = x0;
  a.c0 = c0;
  a.ncols = ncols;
  // columns per workgroup: as many as 64 KB of LDS allows, at most 32
  int nbc = 32;
  while (nbc > 1 && sizeof(double) * (size_t)nb * 2 * C * nbc > 64 * 1024) nbc >>= 1;
  a.nbc = nbc;
  switch (C) {
    case 2: return dispatch<2>(lower, unit, conj, a, s);
    case 3: return dispatch<3>(lower, unit, conj, a, s);
    case 4: return dispatch<4>(lower, unit, conj, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mplu
