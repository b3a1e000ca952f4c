// k_trsm.hip -- solve op(T) X = X for one nb x nb triangular block T, in place, many
// right-hand-side columns at once.
//
// Used for the block row of U in the blocked LU (U12 := L11^-1 A12, Kouya Sec. 3) and for
// the diagonal blocks of the blocked substitutions (Sec. 4).  Each workgroup stages the
// triangle in LDS and sweeps a strip of columns of X, one column per wave and one row
// per lane.  Blocks of more than 64 rows are split in halves around a 4M product.  Element operations use the 4M complex product with one rounding per part
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
  // optional row interchanges to apply to this workgroup's columns first: swl[0] pairs,
  // destination rows at swl + 1, source rows at swl + 1 + swstride (absolute rows of X)
  const int32_t *swl;
  int swstride;
  int urgent;  // raise the waves' issue priority (critical-path solve)
};

// op(T)[r][i]; RE: a real matrix (C planes), op = transpose when CONJ, im returned zero
template <int C, bool CONJ, bool RE>
__device__ __forceinline__ void ld_opT(const TrsmArgs &a, int r, int i, double (&re)[C],
                                       double (&im)[C]) {
  if (RE) {
    if (CONJ) ld_re<C>(a.T, a.t0 + i, a.t0 + r, re);
    else ld_re<C>(a.T, a.t0 + r, a.t0 + i, re);
#pragma unroll
    for (int c = 0; c < C; ++c) im[c] = 0.0;
  } else if (CONJ) {
    ld_z<C>(a.T, a.t0 + i, a.t0 + r, re, im);
#pragma unroll
    for (int c = 0; c < C; ++c) im[c] = -im[c];
  } else {
    ld_z<C>(a.T, a.t0 + r, a.t0 + i, re, im);
  }
}

// value of lane s (s uniform across the wave)
__device__ __forceinline__ double wbcast(double v, int s) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), s);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), s);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// LOWER: op(T) is lower triangular (forward sweep); UNIT: unit diagonal.  nb <= 64.
// The strict triangle of op(T) is staged once in LDS, packed by columns in component
// planes (column i holds rows i+1..nb-1 when LOWER, rows 0..i-1 otherwise), with the
// reciprocals of the diagonal.  Each wave then owns TW right-hand-side columns at a
// time, one row per lane: a step finishes unknown s on lane s, broadcasts it across the
// wave and updates the other rows, with no workgroup barrier inside the sweep.
// RE: real matrices (only the C real planes are read and written), real arithmetic.
template <int C, bool LOWER, bool UNIT, bool CONJ, int TW, bool RE>
__global__ __launch_bounds__(256) void k_trsm(TrsmArgs a) {
  extern __shared__ double smem[];
  if (a.urgent) __builtin_amdgcn_s_setprio(2);
  constexpr int Q = RE ? C : 2 * C;
  // TW: columns per wave in flight (more hides latency, fewer spreads a narrow strip)
  const int nb = a.nb, NBC = a.nbc, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int ntri = nb * (nb - 1) / 2;
  const int64_t cb = a.c0 + (int64_t)blockIdx.x * NBC;
  const int64_t left = a.c0 + a.ncols - cb;
  const int ncl = (int)(left < NBC ? left : NBC);
  double *sR = smem;                    // [Q][nb] reciprocals of the diagonal
  double *sT = sR + (size_t)nb * Q;     // [Q][ntri] packed strict triangle

  auto col_off = [&](int i) { return LOWER ? i * (nb - 1) - i * (i - 1) / 2 : i * (i - 1) / 2; };

  if (a.swl) {
    // row interchanges of this workgroup's columns, one column per wave at a time: every
    // read of a column before any write to it (at most 256 pairs)
    // the count and both halves of the list are read together (the list has swstride
    // slots per half), then masked by the count
    const int cnt = a.swl[0];
    const int32_t *dst = a.swl + 1, *src = a.swl + 1 + a.swstride;
    int32_t sr[4], ds[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int e = lane + 64 * h;
      sr[h] = e < a.swstride ? src[e] : -1;
      ds[h] = e < a.swstride ? dst[e] : -1;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const bool live = lane + 64 * h < cnt;
      sr[h] = live ? sr[h] : -1;
      ds[h] = live ? ds[h] : -1;
    }
    for (int cc = w; cc < ncl; cc += 4) {
      double *col0 = a.X.p + (cb + cc) * a.X.ld;
      double v[4][Q];
#pragma unroll
      for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int q = 0; q < Q; ++q) v[h][q] = sr[h] >= 0 ? col0[(int64_t)q * a.X.ps + sr[h]] : 0.0;
#pragma unroll
      for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (ds[h] >= 0) col0[(int64_t)q * a.X.ps + ds[h]] = v[h][q];
    }
    __syncthreads();
  }

  // strict triangle, column by column: wave w takes columns w, w + 4, ...; lane = row.
  // Eight columns' loads are issued before their LDS stores.
  constexpr int SB = 8;
  for (int i0 = w; i0 < nb; i0 += 4 * SB) {
    double tv[SB][Q];
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int i = i0 + 4 * u;
      const bool in = i < nb && (LOWER ? (lane > i && lane < nb) : (lane < i));
      double tr[C], ti[C];
      if (in) {
        ld_opT<C, CONJ, RE>(a, lane, i, tr, ti);
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) tr[c] = ti[c] = 0.0;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        tv[u][c] = tr[c];
        if (!RE) tv[u][RE ? 0 : C + c] = ti[c];
      }
    }
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int i = i0 + 4 * u;
      const bool in = i < nb && (LOWER ? (lane > i && lane < nb) : (lane < i));
      if (in) {
        const int off = col_off(i) + (LOWER ? lane - i - 1 : lane);
#pragma unroll
        for (int q = 0; q < Q; ++q) sT[(size_t)q * ntri + off] = tv[u][q];
      }
    }
  }
  if (!UNIT) {
    for (int i = t; i < nb; i += 256) {
      double dr[C], di[C], rr[C], ri[C];
      ld_opT<C, CONJ, RE>(a, i, i, dr, di);
      if (RE) mp::recip<C>(dr, rr);
      else mp::zrecip<C>(dr, di, rr, ri);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        sR[c * nb + i] = rr[c];
        if (!RE) sR[(C + c) * nb + i] = ri[c];
      }
    }
  }
  __syncthreads();

  double rr[C], ri[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    rr[c] = (!UNIT && lane < nb) ? sR[c * nb + lane] : 0.0;
    ri[c] = (!RE && !UNIT && lane < nb) ? sR[(C + c) * nb + lane] : 0.0;
  }

  for (int cc0 = w * TW; cc0 < ncl; cc0 += 4 * TW) {
    double xr[TW][C], xi[TW][C];
#pragma unroll
    for (int h = 0; h < TW; ++h) {
      if (RE && lane < nb && cc0 + h < ncl) {
        ld_re<C>(a.X, a.x0 + lane, cb + cc0 + h, xr[h]);
#pragma unroll
        for (int c = 0; c < C; ++c) xi[h][c] = 0.0;
      } else if (lane < nb && cc0 + h < ncl) {
        ld_z<C>(a.X, a.x0 + lane, cb + cc0 + h, xr[h], xi[h]);
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) xr[h][c] = xi[h][c] = 0.0;
      }
    }
    for (int u = 0; u < nb; ++u) {
      const int i = LOWER ? u : nb - 1 - u;
      if (!UNIT && lane == i) {
#pragma unroll
        for (int h = 0; h < TW; ++h) {
          double orr[C], oi[C];
          if (RE) {
            mp::mul<C>(xr[h], rr, orr);
            mp::set_zero<C>(oi);
          } else {
            mp::zmul<C>(xr[h], xi[h], rr, ri, orr, oi);
          }
#pragma unroll
          for (int c = 0; c < C; ++c) {
            xr[h][c] = orr[c];
            xi[h][c] = oi[c];
          }
        }
      }
      const bool upd = LOWER ? (lane > i && lane < nb) : (lane < i);
      const int off = col_off(i) + (LOWER ? lane - i - 1 : lane);
      double tr[C], ti[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        tr[c] = upd ? sT[(size_t)c * ntri + off] : 0.0;
        ti[c] = (!RE && upd) ? sT[(size_t)(RE ? 0 : C + c) * ntri + off] : 0.0;
      }
#pragma unroll
      for (int h = 0; h < TW; ++h) {
        double yr[C], yi[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          yr[c] = wbcast(xr[h][c], i);
          yi[c] = RE ? 0.0 : wbcast(xi[h][c], i);
        }
        if (upd) {
          if (RE) {  // x -= t y
            double l[C], nt[C];
            mp::copy<C>(xr[h], l);
            mp::neg<C>(tr, nt);
            mp::mac<C>(l, nt, yr);
            mp::renorm<C>(l, xr[h]);
          } else {
            mp::zfms<C>(xr[h], xi[h], tr, ti, yr, yi, xr[h], xi[h]);
          }
        }
      }
    }
#pragma unroll
    for (int h = 0; h < TW; ++h)
      if (lane < nb && cc0 + h < ncl) {
        if (RE) st_re<C>(a.X, a.x0 + lane, cb + cc0 + h, xr[h]);
        else st_z<C>(a.X, a.x0 + lane, cb + cc0 + h, xr[h], xi[h]);
      }
  }
}

template <int C, bool LOWER, bool UNIT, bool CONJ, int TW, bool RE>
static hipError_t go_tw(const TrsmArgs &a, hipStream_t s) {
  constexpr int Q = RE ? C : 2 * C;
  const size_t lds = sizeof(double) * ((size_t)a.nb * Q + (size_t)Q * (a.nb * (a.nb - 1) / 2));
  static LdsAttr attr;
  const hipError_t e = attr.ensure((const void *)k_trsm<C, LOWER, UNIT, CONJ, TW, RE>, 160 * 1024);
  if (e != hipSuccess) return e;
  const int64_t blocks = (a.ncols + a.nbc - 1) / a.nbc;
  hipLaunchKernelGGL((k_trsm<C, LOWER, UNIT, CONJ, TW, RE>), dim3((unsigned)blocks), dim3(256),
                     lds, s, a);
  return hipGetLastError();
}

// a strip of 4 columns per workgroup runs one column per wave
template <int C, bool LOWER, bool UNIT, bool CONJ, bool RE>
static hipError_t go(const TrsmArgs &a, hipStream_t s) {
  return a.nbc == 4 ? go_tw<C, LOWER, UNIT, CONJ, 1, RE>(a, s)
                    : go_tw<C, LOWER, UNIT, CONJ, 2, RE>(a, s);
}

template <int C, bool RE>
static hipError_t dispatch(bool lower, bool unit, bool conj, const TrsmArgs &a, hipStream_t s) {
  // op(T) is lower when T is lower and not transposed, or T upper and transposed
  const bool opl = lower != conj;
  if (opl) {
    if (unit) return conj ? go<C, true, true, true, RE>(a, s) : go<C, true, true, false, RE>(a, s);
    return conj ? go<C, true, false, true, RE>(a, s) : go<C, true, false, false, RE>(a, s);
  }
  if (unit) return conj ? go<C, false, true, true, RE>(a, s) : go<C, false, true, false, RE>(a, s);
  return conj ? go<C, false, false, true, RE>(a, s) : go<C, false, false, false, RE>(a, s);
}

hipError_t launch_trsm(int C, bool lower, bool unit, bool conj, ZM Tm, int64_t t0, int nb,
                       ZM Xm, int64_t x0, int64_t c0, int64_t ncols, hipStream_t s,
                       const int32_t *swl, int swstride, bool real, bool urgent) {
  if (nb <= 0 || ncols <= 0) return hipSuccess;
  if (nb > 64) {
    if (swl) {
      hipError_t e = launch_laswp_list(C, Xm, c0, ncols, swl, swstride, s, real);
      if (e != hipSuccess) return e;
    }
    // one row per lane: split op(T) into halves,
    //   lower op:  X1 = T11^-1 X1;  X2 -= T21 X1;  X2 = T22^-1 X2
    //   upper op:  X2 = T22^-1 X2;  X1 -= T12 X2;  X1 = T11^-1 X1
    const int h = nb / 2, r = nb - h;
    const bool opl = lower != conj;
    const char opA = conj ? 'C' : 'N';
    hipError_t e;
    const int gm = real ? 2 : 0;  // the real product, else 4M
    if (opl) {
      if ((e = launch_trsm(C, lower, unit, conj, Tm, t0, h, Xm, x0, c0, ncols, s, nullptr, 0,
                           real)) != hipSuccess)
        return e;
      // T21 = op(T)[h:, :h]: stored at (t0+h, t0) untransposed, else (t0, t0+h) transposed
      if ((e = launch_gemm(C, gm, opA, 'N', r, ncols, h, -1, Tm, conj ? t0 : t0 + h,
                           conj ? t0 + h : t0, Xm, x0, c0, 1, Xm, x0 + h, c0, s)) != hipSuccess)
        return e;
      return launch_trsm(C, lower, unit, conj, Tm, t0 + h, r, Xm, x0 + h, c0, ncols, s, nullptr,
                         0, real);
    }
    if ((e = launch_trsm(C, lower, unit, conj, Tm, t0 + h, r, Xm, x0 + h, c0, ncols, s, nullptr,
                         0, real)) != hipSuccess)
      return e;
    // T12 = op(T)[:h, h:]: stored at (t0, t0+h) untransposed, else (t0+h, t0) transposed
    if ((e = launch_gemm(C, gm, opA, 'N', h, ncols, r, -1, Tm, conj ? t0 + h : t0,
                         conj ? t0 : t0 + h, Xm, x0 + h, c0, 1, Xm, x0, c0, s)) != hipSuccess)
      return e;
    return launch_trsm(C, lower, unit, conj, Tm, t0, h, Xm, x0, c0, ncols, s, nullptr, 0, real);
  }
  TrsmArgs a;
  a.T = Tm;
  a.t0 = t0;
  a.nb = nb;
  a.X = Xm;
  a.x0 = x0;
  a.c0 = c0;
  a.ncols = ncols;
  a.swl = swl;
  a.swstride = swstride;
  a.urgent = urgent ? 1 : 0;
  // columns per workgroup: a multiple of the 8 the four waves take per pass (two columns
  // each), enough to spread over about 512 workgroups (two per CU for double-double);
  // strips of at most 256 columns take 4 columns per workgroup, one per wave
  int64_t nbc = (a.ncols + 511) / 512;
  nbc = (nbc + 7) / 8 * 8;
  a.nbc = (int)(nbc < 8 ? 8 : nbc);
  if (a.ncols <= 256) a.nbc = 4;
  switch (C) {
    case 2: return real ? dispatch<2, true>(lower, unit, conj, a, s) : dispatch<2, false>(lower, unit, conj, a, s);
    case 3: return real ? dispatch<3, true>(lower, unit, conj, a, s) : dispatch<3, false>(lower, unit, conj, a, s);
    case 4: return real ? dispatch<4, true>(lower, unit, conj, a, s) : dispatch<4, false>(lower, unit, conj, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mplu
