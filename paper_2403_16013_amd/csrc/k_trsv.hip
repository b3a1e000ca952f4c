// k_trsv.hip -- forward or backward substitution op(T) X = B for a few right-hand sides
// in a single launch (Kouya Sec. 4: the substitutions that follow the LU factorisation).
//
// With one or a handful of right-hand sides a substitution is a chain of n dependent
// steps and almost no arithmetic, so a blocked sweep of separate kernels spends its time
// in launch and drain latency.  Here one launch covers the whole triangle: workgroup
// (q, g) owns block row q (64 rows, one per lane of wave 0) for right-hand-side group g.
// It waits for the blocks it depends on in dependency order, as each one is published,
// and folds its contribution into per-thread level accumulators (the four waves split
// the 64 columns of each block); then wave 0 merges the partial sums into its rows and
// solves the diagonal block one step per row, broadcasting each finished unknown across
// the wave, while the other waves stage the next columns of the diagonal block in LDS.
// The finished block is published with device-coherent stores followed by its ready
// word.  Workgroups only wait on workgroups with lower indices, which are dispatched
// first, so the chain always progresses; every wait is still bounded and an expired wait
// turns the solution into NaN rather than hanging.
//
// Element operations: the 4M complex product (Eq. 4m); a non-unit diagonal is applied by
// its reciprocal, to the rows of the block and of the right-hand side before the sweep.
#include "common.hpp"

#pragma clang fp contract(off)

namespace mplu {

static constexpr int SVB = 64;   // rows per block row
static constexpr int SVCH = 8;   // diagonal-block columns per staged chunk
static constexpr unsigned SV_SPIN_LIMIT = 1u << 26;

struct SvArgs {
  ZM T, X;
  int64_t n, nrhs;
  int nblk, ngrp;
  int32_t *flags;  // [nblk * ngrp] ready words, then one sticky expiry word
};

// op(T)[r][c]; RE: a real matrix (C planes), op = transpose when CONJ, im returned zero
template <int C, bool CONJ, bool RE>
__device__ __forceinline__ void ld_op(const ZM &T, int64_t r, int64_t c, double (&re)[C],
                                      double (&im)[C]) {
  if (RE) {
    if (CONJ) ld_re<C>(T, c, r, re);
    else ld_re<C>(T, r, c, re);
#pragma unroll
    for (int k = 0; k < C; ++k) im[k] = 0.0;
  } else if (CONJ) {
    ld_z<C>(T, c, r, re, im);
#pragma unroll
    for (int k = 0; k < C; ++k) im[k] = -im[k];
  } else {
    ld_z<C>(T, r, c, re, im);
  }
}

__device__ __forceinline__ double sv_get(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void sv_put(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// value of lane s (s uniform across the wave)
__device__ __forceinline__ double bcast(double v, int s) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), s);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), s);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// LOWER: op(T) lower triangular (forward sweep), else upper (backward sweep);
// UNIT: unit diagonal; CONJ: op(T) = T^H; NR: right-hand sides per group.
// RE: real matrices (only the C real planes are read and written), real arithmetic.
template <int C, bool LOWER, bool UNIT, bool CONJ, int NR, bool RE>
__global__ __launch_bounds__(256) void k_trsv(SvArgs a) {
  constexpr int Q = RE ? C : 2 * C;
  constexpr int CI = RE ? 0 : C;  // plane offset of the imaginary part (unused when RE)
  extern __shared__ double smem[];
  double *sx = smem;                          // [Q][NR][SVB]   published block being folded
  double *sp = sx + Q * NR * SVB;             // [4][Q][NR][SVB] per-wave partial sums
  double *sd = sp + 4 * Q * NR * SVB;         // [2][Q][SVCH][SVB] diagonal-block chunks
  double *sRc = sd + 2 * Q * SVCH * SVB;      // [Q][SVB] reciprocals of the diagonal
  __shared__ int s_expired;

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nblk = a.nblk, ngrp = a.ngrp;
  const int qi = blockIdx.x / ngrp, grp = blockIdx.x % ngrp;
  const int ib = LOWER ? qi : nblk - 1 - qi;
  const int64_t n = a.n;
  const int64_t r0 = (int64_t)ib * SVB;
  const int nr = (int)((n - r0) < SVB ? (n - r0) : SVB);
  const int64_t x0 = (int64_t)grp * NR;
  const int ncr = (int)((a.nrhs - x0) < NR ? (a.nrhs - x0) : NR);
  int32_t *ready = a.flags;
  int32_t *expiry = a.flags + (size_t)nblk * ngrp;
  const ZM T = a.T, X = a.X;
  const int nchunk = (nr + SVCH - 1) / SVCH;

  // step u of the diagonal solve handles column col_of(u) of the block
  auto col_of = [&](int u) { return LOWER ? u : nr - 1 - u; };
  auto stage_chunk = [&](int c, int buf, int tid, int nthr) {
    double *dst = sd + (size_t)buf * Q * SVCH * SVB;
    for (int e = tid; e < SVCH * SVB; e += nthr) {
      const int row = e % SVB, uu = e / SVB;
      const int u = c * SVCH + uu;
      double re[C], im[C];
      if (row < nr && u < nr) {
        ld_op<C, CONJ, RE>(T, r0 + row, r0 + col_of(u), re, im);
        if (!UNIT) {
          // row `row` of the block divided by its diagonal entry (by its reciprocal)
          double rr[C], ri[C], orr[C], oi[C];
#pragma unroll
          for (int k = 0; k < C; ++k) {
            rr[k] = sRc[k * SVB + row];
            ri[k] = RE ? 0.0 : sRc[(CI + k) * SVB + row];
          }
          if (RE) {
            mp::mul<C>(re, rr, orr);
            mp::set_zero<C>(oi);
          } else {
            mp::zmul<C>(re, im, rr, ri, orr, oi);
          }
#pragma unroll
          for (int k = 0; k < C; ++k) {
            re[k] = orr[k];
            im[k] = oi[k];
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < C; ++k) re[k] = im[k] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < C; ++k) {
        dst[((size_t)k * SVCH + uu) * SVB + row] = re[k];
        if (!RE) dst[((size_t)(CI + k) * SVCH + uu) * SVB + row] = im[k];
      }
    }
  };

  if (t == 0) s_expired = 0;
  // Non-unit diagonal: every row of the block is divided by its diagonal entry up front
  // (the staged block and, once formed, the right-hand side), so the sweep below needs no
  // division on its chain of dependent steps.
  if (!UNIT) {
    if (w == 0 && lane < nr) {
      double dr[C], di[C], rr[C], ri[C];
      ld_op<C, CONJ, RE>(T, r0 + lane, r0 + lane, dr, di);
      if (RE) mp::recip<C>(dr, rr);
      else mp::zrecip<C>(dr, di, rr, ri);
#pragma unroll
      for (int k = 0; k < C; ++k) {
        sRc[k * SVB + lane] = rr[k];
        if (!RE) sRc[(CI + k) * SVB + lane] = ri[k];
      }
    }
    __syncthreads();
  }
  stage_chunk(0, 0, t, 256);

  // ---- contributions of the blocks this one depends on
  double accR[NR][C], accI[NR][C];
#pragma unroll
  for (int h = 0; h < NR; ++h)
#pragma unroll
    for (int k = 0; k < C; ++k) accR[h][k] = accI[h][k] = 0.0;

  // Each wave folds 16 columns of every block it depends on.  The matrix entries do not
  // depend on the solution, so a batch of them is loaded before the wait for the block's
  // ready word; their latency hides behind the wait.
  constexpr int TB = (C == 2) ? 16 : 8;  // columns per batch (registers)
  const int ndep = LOWER ? ib : nblk - 1 - ib;
  for (int st = 0; st < ndep; ++st) {
    const int jb = LOWER ? st : nblk - 1 - st;
    const int64_t j0 = (int64_t)jb * SVB;
    const int nj = (int)((n - j0) < SVB ? (n - j0) : SVB);
    const int cbeg = w * (SVB / 4);
#pragma unroll
    for (int half = 0; half < (SVB / 4) / TB; ++half) {
      double tv[TB][Q];
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int col = cbeg + half * TB + u;
        double tr[C], ti[C];
        if (lane < nr && col < nj) {
          ld_op<C, CONJ, RE>(T, r0 + lane, j0 + col, tr, ti);
        } else {
#pragma unroll
          for (int k = 0; k < C; ++k) tr[k] = ti[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < C; ++k) {
          tv[u][k] = tr[k];
          if (!RE) tv[u][CI + k] = ti[k];
        }
      }
      if (half == 0) {
        if (t == 0) {
          const int32_t *f = ready + (size_t)jb * ngrp + grp;
          unsigned spins = 0;
          while (__hip_atomic_load(const_cast<int32_t *>(f), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) == 0) {
            if ((spins & 255u) == 255u &&
                __hip_atomic_load(expiry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
              s_expired = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            if (++spins > SV_SPIN_LIMIT) {
              __hip_atomic_store(expiry, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              s_expired = 1;
              break;
            }
          }
        }
        __syncthreads();
        if (!s_expired) {
          for (int e = t; e < Q * NR * SVB; e += 256) {
            const int row = e % SVB, rest = e / SVB, h = rest % NR, q = rest / NR;
            sx[e] = (row < nj && h < ncr)
                        ? sv_get(X.p + (int64_t)q * X.ps + (x0 + h) * X.ld + j0 + row)
                        : 0.0;
          }
        }
        __syncthreads();
      }
      if (s_expired) break;
      if (lane < nr) {
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          const int col = cbeg + half * TB + u;
          if (col < nj) {
            double tr[C], ti[C], ntr[C], nti[C];
#pragma unroll
            for (int k = 0; k < C; ++k) {
              tr[k] = tv[u][k];
              ti[k] = RE ? 0.0 : tv[u][CI + k];
              ntr[k] = -tr[k];
              nti[k] = -ti[k];
            }
#pragma unroll
            for (int h = 0; h < NR; ++h) {
              double xr[C], xi[C];
#pragma unroll
              for (int k = 0; k < C; ++k) {
                xr[k] = sx[((size_t)k * NR + h) * SVB + col];
                xi[k] = RE ? 0.0 : sx[((size_t)(CI + k) * NR + h) * SVB + col];
              }
              // acc -= t x
              mp::mac<C>(accR[h], ntr, xr);
              if (!RE) {
                mp::mac<C>(accR[h], ti, xi);
                mp::mac<C>(accI[h], ntr, xi);
                mp::mac<C>(accI[h], nti, xr);
              }
            }
          }
        }
      }
    }
    if (s_expired) break;
    if (lane < nr) {
      // keep the accumulators non-overlapping between blocks
#pragma unroll
      for (int h = 0; h < NR; ++h) {
        double vr[C], vi[C];
        mp::renorm<C>(accR[h], vr);
        mp::renorm<C>(accI[h], vi);
#pragma unroll
        for (int k = 0; k < C; ++k) {
          accR[h][k] = vr[k];
          accI[h][k] = vi[k];
        }
      }
    }
    __syncthreads();
  }

  // ---- merge the partial sums into the right-hand side (wave 0 owns the rows)
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    double pr[C], pi[C];
    mp::renorm<C>(accR[h], pr);
    mp::renorm<C>(accI[h], pi);
#pragma unroll
    for (int k = 0; k < C; ++k) {
      sp[(((size_t)w * Q + k) * NR + h) * SVB + lane] = pr[k];
      if (!RE) sp[(((size_t)w * Q + CI + k) * NR + h) * SVB + lane] = pi[k];
    }
  }
  __syncthreads();

  double yr[NR][C], yi[NR][C];
  if (w == 0) {
#pragma unroll
    for (int h = 0; h < NR; ++h) {
      double lr[C], li[C];
      if (RE && lane < nr && h < ncr) {
        ld_re<C>(X, r0 + lane, x0 + h, lr);
#pragma unroll
        for (int k = 0; k < C; ++k) li[k] = 0.0;
      } else if (lane < nr && h < ncr) {
        ld_z<C>(X, r0 + lane, x0 + h, lr, li);
      } else {
#pragma unroll
        for (int k = 0; k < C; ++k) lr[k] = li[k] = 0.0;
      }
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        double vr[C], vi[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
          vr[k] = sp[(((size_t)ww * Q + k) * NR + h) * SVB + lane];
          vi[k] = RE ? 0.0 : sp[(((size_t)ww * Q + CI + k) * NR + h) * SVB + lane];
        }
        mp::push_mp<C>(lr, vr);
        if (!RE) mp::push_mp<C>(li, vi);
      }
      mp::renorm<C>(lr, yr[h]);
      mp::renorm<C>(li, yi[h]);
      if (!UNIT && lane < nr) {
        double rr[C], ri[C], orr[C], oi[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
          rr[k] = sRc[k * SVB + lane];
          ri[k] = RE ? 0.0 : sRc[(CI + k) * SVB + lane];
        }
        if (RE) {
          mp::mul<C>(yr[h], rr, orr);
          mp::set_zero<C>(oi);
        } else {
          mp::zmul<C>(yr[h], yi[h], rr, ri, orr, oi);
        }
#pragma unroll
        for (int k = 0; k < C; ++k) {
          yr[h][k] = orr[k];
          yi[h][k] = oi[k];
        }
      }
    }
  }

  // ---- diagonal block: one step per row on wave 0, next chunk staged by waves 1-3
  for (int c = 0; c < nchunk; ++c) {
    if (w == 0) {
      const double *ch = sd + (size_t)(c & 1) * Q * SVCH * SVB;
      const int ucount = (nr - c * SVCH) < SVCH ? nr - c * SVCH : SVCH;
      for (int uu = 0; uu < ucount; ++uu) {
        const int s = col_of(c * SVCH + uu);
        double tr[C], ti[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
          tr[k] = ch[((size_t)k * SVCH + uu) * SVB + lane];
          ti[k] = RE ? 0.0 : ch[((size_t)(CI + k) * SVCH + uu) * SVB + lane];
        }
        const bool upd = lane < nr && (LOWER ? lane > s : lane < s);
#pragma unroll
        for (int h = 0; h < NR; ++h) {
          double xr[C], xi[C];
#pragma unroll
          for (int k = 0; k < C; ++k) {
            xr[k] = bcast(yr[h][k], s);
            xi[k] = RE ? 0.0 : bcast(yi[h][k], s);
          }
          if (upd) {
            if (RE) {  // y -= t x
              double l[C], nt[C];
              mp::copy<C>(yr[h], l);
              mp::neg<C>(tr, nt);
              mp::mac<C>(l, nt, xr);
              mp::renorm<C>(l, yr[h]);
            } else {
              mp::zfms<C>(yr[h], yi[h], tr, ti, xr, xi, yr[h], yi[h]);
            }
          }
        }
      }
    } else if (c + 1 < nchunk) {
      stage_chunk(c + 1, (c + 1) & 1, t - 64, 192);
    }
    __syncthreads();
  }

  // ---- publish the block, then its ready word
  if (w == 0) {
    const bool bad = s_expired != 0;
    if (lane < nr) {
#pragma unroll
      for (int h = 0; h < NR; ++h) {
        if (h < ncr) {
          double *b = X.p + (x0 + h) * X.ld + r0 + lane;
#pragma unroll
          for (int k = 0; k < C; ++k) {
            sv_put(b + (int64_t)k * X.ps, bad ? __builtin_nan("") : yr[h][k]);
            if (!RE) sv_put(b + (int64_t)(C + k) * X.ps, bad ? __builtin_nan("") : yi[h][k]);
          }
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    if (lane == 0)
      __hip_atomic_store(ready + (size_t)ib * ngrp + grp, 1, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int C, bool LOWER, bool UNIT, bool CONJ, int NR, bool RE>
static hipError_t go_sv(const SvArgs &a, hipStream_t s) {
  constexpr int Q = RE ? C : 2 * C;
  const size_t lds =
      sizeof(double) * ((size_t)5 * Q * NR * SVB + (size_t)2 * Q * SVCH * SVB + (size_t)Q * SVB);
  static LdsAttr attr;
  const hipError_t e = attr.ensure((const void *)k_trsv<C, LOWER, UNIT, CONJ, NR, RE>, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_trsv<C, LOWER, UNIT, CONJ, NR, RE>), dim3((unsigned)(a.nblk * a.ngrp)),
                     dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int C, int NR, bool RE>
static hipError_t dispatch_sv(bool lower, bool unit, bool conj, const SvArgs &a, hipStream_t s) {
  // op(T) is lower when T is lower and not transposed, or T upper and transposed
  const bool opl = lower != conj;
  if (opl) {
    if (unit) return conj ? go_sv<C, true, true, true, NR, RE>(a, s) : go_sv<C, true, true, false, NR, RE>(a, s);
    return conj ? go_sv<C, true, false, true, NR, RE>(a, s) : go_sv<C, true, false, false, NR, RE>(a, s);
  }
  if (unit) return conj ? go_sv<C, false, true, true, NR, RE>(a, s) : go_sv<C, false, true, false, NR, RE>(a, s);
  return conj ? go_sv<C, false, false, true, NR, RE>(a, s) : go_sv<C, false, false, false, NR, RE>(a, s);
}

static inline int sv_nr(int64_t nrhs) { return nrhs >= 3 ? 4 : (int)nrhs; }

int64_t trsv_flag_words(int64_t n, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return 1;
  const int NR = sv_nr(nrhs);
  return ((n + SVB - 1) / SVB) * ((nrhs + NR - 1) / NR) + 1;
}

hipError_t launch_trsv(int C, bool lower, bool unit, bool conj, ZM Tm, ZM Xm, int64_t n,
                       int64_t nrhs, int32_t *flags, hipStream_t s, bool real) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  const int NR = sv_nr(nrhs);
  SvArgs a;
  a.T = Tm;
  a.X = Xm;
  a.n = n;
  a.nrhs = nrhs;
  a.nblk = (int)((n + SVB - 1) / SVB);
  a.ngrp = (int)((nrhs + NR - 1) / NR);
  a.flags = flags;
  hipError_t e = launch_fill_i32(flags, 0, trsv_flag_words(n, nrhs), s);
  if (e != hipSuccess) return e;
#define SV_NR(CC)                                                                    \
  switch (NR) {                                                                      \
    case 1: return real ? dispatch_sv<CC, 1, true>(lower, unit, conj, a, s)          \
                        : dispatch_sv<CC, 1, false>(lower, unit, conj, a, s);        \
    case 2: return real ? dispatch_sv<CC, 2, true>(lower, unit, conj, a, s)          \
                        : dispatch_sv<CC, 2, false>(lower, unit, conj, a, s);        \
    default: return real ? dispatch_sv<CC, 4, true>(lower, unit, conj, a, s)         \
                         : dispatch_sv<CC, 4, false>(lower, unit, conj, a, s);       \
  }
  switch (C) {
    case 2: SV_NR(2)
    case 3: SV_NR(3)
    case 4: SV_NR(4)
  }
#undef SV_NR
  return hipErrorInvalidValue;
}

}  // namespace mplu
