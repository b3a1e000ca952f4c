// k_gemm.hip -- complex multi-component matrix product
//     Cm := beta*Cm + alpha * op(A) * op(B)
// by the 4M method (Kouya Eq. 4m) or the 3M method (Eq. 3m_cemm).  This is the trailing
// update A22 -= L21 U12 of the blocked LU (Sec. 3), where nearly all the time goes.
//
// Design for gfx950: the product is bound by FP64 vector arithmetic (each complex MAC is
// 36 (3M, DD; 30 when its cross products run on the matrix cores, see XM below) to ~350
// (3M, QD) FP64 instructions), so the kernel is a classic LDS-tiled
// register-blocked GEMM: a workgroup owns a BM x BN output tile, stages BK-deep slabs of
// op(A) and op(B) in LDS (for 3M together with the rounded sums Re+Im of Eq. 3m_cemm,
// computed once per staged element), and each thread accumulates a TM x TN micro-tile in
// level accumulators (see mp.hpp).  3M keeps T1 = ReA ReB, T2 = ImA ImB and
// T3 = (ReA+ImA)(ReB+ImB) apart over the whole K range and combines them in the
// epilogue: Re = T1 - T2, Im = T3 - T1 - T2, added to Cm with a single rounding per part.
// 4M accumulates straight into Cm's value (alpha folded into the staged A).
#include <stdlib.h>

#include "common.hpp"

#pragma clang fp contract(off)

namespace mplu {

struct GemmArgs {
  ZM A, B, Cm;
  int64_t ai, aj, bi, bj, ci, cj;
  int64_t m, n, k;
  int opA, opB;  // 'N', 'T', 'C'
  int alpha, beta;
  int urgent;  // raise the waves' issue priority (critical-path product)
};

// Products deeper than TIDY_MIN_K (never the trailing updates of the factorisation, whose
// depth is the panel width) re-level their accumulators (mp::tidy) after every TIDY_K
// steps of k.  Without it the error of a long sum of same-sign products grows faster than
// k u for C >= 3 (a host measurement at k = 4096, uniform [0, 1] data: about 10^4 u for
// QD, against 15 u with re-levelling every 16 steps).
constexpr int TIDY_K = 16;
constexpr int64_t TIDY_MIN_K = 128;

// RE: the real product (the Im = 0 case of the 3M form: only T1 = ReA ReB is formed,
// only the real planes are read and written; the imaginary planes are never touched).
// Waves per SIMD asked of the compiler for the 32 x 32 3M tiles: three for double-double
// with the cross products on the matrix cores (XM, every trailing update) and four
// without them (longer products, 128 registers); three for triple-double, where a few
// address values then live in scratch and are reloaded once per staged slab, never inside
// the k loop.  Measured 1-4% faster on the trailing update than the waves the register use
// would otherwise give.  Quadruple-double stays at two (three would spill inside the k
// loop).
template <int C, bool M3, int BM, int BN, int BK, int UNR, bool RE, bool XM = false>
constexpr int gemm_min_waves() {
  if (BM != 32 || BN != 32 || BK != 8 || RE || !M3) return 1;
  if (XM) return 3;  // the MFMA cross accumulators need 10 more registers
  return C == 2 ? (UNR == 2 ? 4 : 1) : (C == 3 ? 3 : 1);
}

// The double-double MAC of mp::mac without its two cross products a_hi b_lo + a_lo b_hi:
// TwoProd of the leading parts, its product into level 0 by TwoSum, both errors into
// level 1 (10 instructions instead of 12).  The cross products, needed to binary64
// accuracy only (level-1 terms), are summed separately on the FP64 matrix cores.
__device__ __forceinline__ void mac_dd_lead(double (&l)[2], const double (&a)[2],
                                            const double (&b)[2]) {
  double p, e, s, t;
  mp::two_prod(a[0], b[0], p, e);
  mp::two_sum(l[0], p, s, t);
  l[0] = s;
  l[1] += t;
  l[1] += e;
}

// XM: double-double 3M or real products of depth <= TIDY_MIN_K with the cross products on
// v_mfma_f64_16x16x4f64.  Every 16 x 16 block of the output is summed over k in the same
// 4-deep steps, (a_hi b_lo) then (a_lo b_hi) in each, in both tilings: in 32 x 32 tiles
// each wave owns one 16 x 16 quarter for all NV products; in 16 x 16 tiles wave v owns
// product v.  The sums reach level 1 of the accumulators once, after the last step of k.
// On this GPU the FP64 matrix rate equals the vector rate, so the gain is the issue slots
// of the two FMAs (first trailing update at n = 4096, K = 64: 1.75 -> 1.70 ms).  The 32 x 32
// tiles run three waves per SIMD: at four, a cross accumulator went to scratch for every
// slab (1% faster, but 60% more bytes written to memory).
template <int C, bool M3, int BM, int BN, int BK, int TM, int TN, int UNR, bool RE = false,
          bool XM = false>
__global__ __launch_bounds__((BM / TM) * (BN / TN), (gemm_min_waves<C, M3, BM, BN, BK, UNR, RE, XM>()))
void k_gemm(GemmArgs g) {
  if (g.urgent) __builtin_amdgcn_s_setprio(2);
  constexpr int NT = (BM / TM) * (BN / TN);
  constexpr int NV = RE ? 1 : (M3 ? 3 : 2);
  constexpr int SX = BN / TN;  // threads along n
  constexpr int SY = BM / TM;  // threads along m
  static_assert(TIDY_K % BK == 0, "re-levelling points must fall on slab ends");
  static_assert(!XM || (C == 2 && (M3 || RE) && NT == 256 && BK % 4 == 0 &&
                        ((BM == 32 && BN == 32) || (BM == 16 && BN == 16))),
                "cross products on the matrix cores: double-double 3M / real, 16 or 32 tiles");
  __shared__ double sA[BK][NV][C][BM];
  __shared__ double sB[BK][NV][C][BN];
  typedef double v4d __attribute__((ext_vector_type(4)));
  // 16 x 16 blocks per wave and their products: 32 x 32 tiles, quarter w, all NV
  // products; 16 x 16 tiles, wave v < NV, product v
  constexpr int XN = (BM == 32) ? NV : 1;
  v4d xacc[XN];
#pragma unroll
  for (int q = 0; q < XN; ++q) xacc[q] = v4d{0.0, 0.0, 0.0, 0.0};

  const int tid = threadIdx.x;
  const int tx = tid % SX, ty = tid / SX;
  int64_t tm, tn;
  xcd_tile((g.m + BM - 1) / BM, (g.n + BN - 1) / BN, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;

  // accumulators
  double acc[NV][TM][TN][C];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int jj = 0; jj < TN; ++jj)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[v][i][jj][c] = 0.0;

  if (!M3 && !RE && g.beta) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int jj = 0; jj < TN; ++jj) {
        const int64_t mi = m0 + ty + i * SY, nj = n0 + tx + jj * SX;
        if (mi < g.m && nj < g.n) {
          double re[C], im[C];
          ld_z<C>(g.Cm, g.ci + mi, g.cj + nj, re, im);
#pragma unroll
          for (int c = 0; c < C; ++c) {
            acc[0][i][jj][c] = re[c];
            acc[1][i][jj][c] = im[c];
          }
        }
      }
  }

  const double asign = (!M3 && !RE && g.alpha < 0) ? -1.0 : 1.0;

  for (int64_t k0 = 0; k0 < g.k; k0 += BK) {
    // the staging addresses are recomputed for every slab from an opaque copy of the
    // thread index: kept live across the k loop instead, they would be spilled to scratch
    // at the register budget the launch bounds ask for
    int tids = tid;
    if (gemm_min_waves<C, M3, BM, BN, BK, UNR, RE, XM>() > 1) asm volatile("" : "+v"(tids));
    // stage op(A)[m0 .. m0+BM) x [k0 .. k0+BK)
    for (int e = tids; e < BM * BK; e += NT) {
      int mm, kk;
      if (g.opA == 'N') { mm = e % BM; kk = e / BM; }
      else { kk = e % BK; mm = e / BK; }
      const int64_t gi = m0 + mm, gt = k0 + kk;
      double re[C], im[C];
      if (RE && gi < g.m && gt < g.k) {
        if (g.opA == 'N') ld_re<C>(g.A, g.ai + gi, g.aj + gt, re);
        else ld_re<C>(g.A, g.ai + gt, g.aj + gi, re);
      } else if (gi < g.m && gt < g.k) {
        if (g.opA == 'N') ld_z<C>(g.A, g.ai + gi, g.aj + gt, re, im);
        else ld_z<C>(g.A, g.ai + gt, g.aj + gi, re, im);
        const double isg = (g.opA == 'C') ? -asign : asign;
#pragma unroll
        for (int c = 0; c < C; ++c) { re[c] *= asign; im[c] *= isg; }
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) { re[c] = 0.0; im[c] = 0.0; }
      }
      if (RE) {
#pragma unroll
        for (int c = 0; c < C; ++c) sA[kk][0][c][mm] = re[c];
        continue;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) { sA[kk][0][c][mm] = re[c]; sA[kk][1][c][mm] = im[c]; }
      if (M3) {
        double s[C];
        mp::add<C>(re, im, s);
#pragma unroll
        for (int c = 0; c < C; ++c) sA[kk][NV - 1][c][mm] = s[c];
      }
    }
    // stage op(B)[k0 .. k0+BK) x [n0 .. n0+BN)
    for (int e = tids; e < BN * BK; e += NT) {
      int nn, kk;
      if (g.opB == 'N') { kk = e % BK; nn = e / BK; }
      else { nn = e % BN; kk = e / BN; }
      const int64_t gj = n0 + nn, gt = k0 + kk;
      double re[C], im[C];
      if (RE && gj < g.n && gt < g.k) {
        if (g.opB == 'N') ld_re<C>(g.B, g.bi + gt, g.bj + gj, re);
        else ld_re<C>(g.B, g.bi + gj, g.bj + gt, re);
      } else if (gj < g.n && gt < g.k) {
        if (g.opB == 'N') ld_z<C>(g.B, g.bi + gt, g.bj + gj, re, im);
        else ld_z<C>(g.B, g.bi + gj, g.bj + gt, re, im);
        if (g.opB == 'C') {
#pragma unroll
          for (int c = 0; c < C; ++c) im[c] = -im[c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) { re[c] = 0.0; im[c] = 0.0; }
      }
      if (RE) {
#pragma unroll
        for (int c = 0; c < C; ++c) sB[kk][0][c][nn] = re[c];
        continue;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) { sB[kk][0][c][nn] = re[c]; sB[kk][1][c][nn] = im[c]; }
      if (M3) {
        double s[C];
        mp::add<C>(re, im, s);
#pragma unroll
        for (int c = 0; c < C; ++c) sB[kk][NV - 1][c][nn] = s[c];
      }
    }
    __syncthreads();

    if constexpr (XM) {
      const int w = tid >> 6, lane = tid & 63;
      const int xr = (BM == 32) ? 16 * (w >> 1) : 0, xc = (BM == 32) ? 16 * (w & 1) : 0;
      if (BM == 32 || w < NV) {
#pragma unroll
        for (int st = 0; st < BK / 4; ++st) {
          const int kq = 4 * st + (lane >> 4);
#pragma unroll
          for (int q = 0; q < XN; ++q) {
            const int v = (BM == 32) ? q : w;
            const double ah = sA[kq][v][0][xr + (lane & 15)], al = sA[kq][v][1][xr + (lane & 15)];
            const double bh = sB[kq][v][0][xc + (lane & 15)], bl = sB[kq][v][1][xc + (lane & 15)];
            xacc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ah, bl, xacc[q], 0, 0, 0);
            xacc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(al, bh, xacc[q], 0, 0, 0);
          }
        }
      }
    }

#pragma unroll UNR
    for (int kk = 0; kk < BK; ++kk) {
      double a[NV][TM][C], b[NV][TN][C];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int c = 0; c < C; ++c) a[v][i][c] = sA[kk][v][c][ty + i * SY];
#pragma unroll
        for (int jj = 0; jj < TN; ++jj)
#pragma unroll
          for (int c = 0; c < C; ++c) b[v][jj][c] = sB[kk][v][c][tx + jj * SX];
      }
      if constexpr (XM) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int jj = 0; jj < TN; ++jj)
#pragma unroll
            for (int v = 0; v < NV; ++v) mac_dd_lead(acc[v][i][jj], a[v][i], b[v][jj]);
      } else if (RE) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int jj = 0; jj < TN; ++jj) mp::mac<C>(acc[0][i][jj], a[0][i], b[0][jj]);
      } else if (M3) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int jj = 0; jj < TN; ++jj) {
            mp::mac<C>(acc[0][i][jj], a[0][i], b[0][jj]);
            mp::mac<C>(acc[1][i][jj], a[1][i], b[1][jj]);
            mp::mac<C>(acc[NV - 1][i][jj], a[NV - 1][i], b[NV - 1][jj]);
          }
      } else {
        double na[TM][C];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int c = 0; c < C; ++c) na[i][c] = -a[1][i][c];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int jj = 0; jj < TN; ++jj) {
            mp::mac<C>(acc[0][i][jj], a[0][i], b[0][jj]);
            mp::mac<C>(acc[0][i][jj], na[i], b[1][jj]);
            mp::mac<C>(acc[1][i][jj], a[0][i], b[1][jj]);
            mp::mac<C>(acc[1][i][jj], a[1][i], b[0][jj]);
          }
      }
    }
    // long products re-level the accumulators every TIDY_K steps of k (counted from the
    // first, at the same k in every kernel so that the tiling never changes a result)
    if (g.k > TIDY_MIN_K && ((k0 + BK) % TIDY_K) == 0 && k0 + BK <= g.k) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int jj = 0; jj < TN; ++jj) mp::tidy<C>(acc[v][i][jj]);
    }
    __syncthreads();
  }

  if constexpr (XM) {
    // the cross sums to level 1 of their elements' accumulators, through LDS (the staging
    // buffers, free after the last slab): X[v][row][col] at v BM BN + row BN + col
    constexpr int NA = BK * NV * C * BM;
    static_assert(NA + BK * NV * C * BN >= NV * BM * BN, "exchange fits the staging buffers");
    double *fa = &sA[0][0][0][0], *fb = &sB[0][0][0][0];
    auto X = [&](int idx) -> double & { return idx < NA ? fa[idx] : fb[idx - NA]; };
    const int w = tid >> 6, lane = tid & 63;
    const int xr = (BM == 32) ? 16 * (w >> 1) : 0, xc = (BM == 32) ? 16 * (w & 1) : 0;
    if (BM == 32 || w < NV) {
#pragma unroll
      for (int q = 0; q < XN; ++q) {
        const int v = (BM == 32) ? q : w;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          X(v * BM * BN + (xr + 4 * e + (lane >> 4)) * BN + xc + (lane & 15)) = xacc[q][e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int jj = 0; jj < TN; ++jj)
          acc[v][i][jj][1] += X(v * BM * BN + (ty + i * SY) * BN + tx + jj * SX);
  }

  // epilogue
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int jj = 0; jj < TN; ++jj) {
      const int64_t mi = m0 + ty + i * SY, nj = n0 + tx + jj * SX;
      if (mi >= g.m || nj >= g.n) continue;
      double ore[C], oim[C];
      if (RE) {
        // the real part of the 3M epilogue with T2 = 0 and the imaginary part left alone
        double t1[C], lr[C];
        mp::renorm<C>(acc[0][i][jj], t1);
        if (g.alpha < 0) mp::neg<C>(t1, t1);
        if (g.beta) ld_re<C>(g.Cm, g.ci + mi, g.cj + nj, lr);
        else mp::set_zero<C>(lr);
        mp::push_mp<C>(lr, t1);
        mp::renorm<C>(lr, ore);
        st_re<C>(g.Cm, g.ci + mi, g.cj + nj, ore);
        continue;
      }
      if (M3) {
        double t1[C], t2[C], t3[C];
        mp::renorm<C>(acc[0][i][jj], t1);
        mp::renorm<C>(acc[1][i][jj], t2);
        mp::renorm<C>(acc[NV - 1][i][jj], t3);
        if (g.alpha < 0) {
          mp::neg<C>(t1, t1);
          mp::neg<C>(t2, t2);
          mp::neg<C>(t3, t3);
        }
        double lr[C], li[C];
        if (g.beta) {
          ld_z<C>(g.Cm, g.ci + mi, g.cj + nj, lr, li);
        } else {
          mp::set_zero<C>(lr);
          mp::set_zero<C>(li);
        }
        mp::push_mp<C>(lr, t1);
        mp::push_mp_neg<C>(lr, t2);
        mp::push_mp<C>(li, t3);
        mp::push_mp_neg<C>(li, t1);
        mp::push_mp_neg<C>(li, t2);
        mp::renorm<C>(lr, ore);
        mp::renorm<C>(li, oim);
      } else {
        mp::renorm<C>(acc[0][i][jj], ore);
        mp::renorm<C>(acc[1][i][jj], oim);
      }
      st_z<C>(g.Cm, g.ci + mi, g.cj + nj, ore, oim);
    }
}

// Narrow products (n <= 16 output columns, 4M): the block updates of the forward and
// backward substitutions.  One thread per output element; op(B) is staged in LDS in
// 32-deep chunks, op(A) is read straight from global memory (each row by n neighbouring
// threads).  Accumulation is the same 4M level accumulation as k_gemm.
template <int C>
__global__ __launch_bounds__(256) void k_gemm_narrow(GemmArgs g, int npow) {
  constexpr int KC = 32;
  __shared__ double sB[KC][2][C][16];
  const int t = threadIdx.x;
  const int rows_per_block = 256 / npow;
  const int64_t mi = (int64_t)blockIdx.x * rows_per_block + t / npow;
  const int nj = t % npow;
  const bool live = (mi < g.m) && (nj < g.n);
  double acr[C], aci[C];
  mp::set_zero<C>(acr);
  mp::set_zero<C>(aci);
  if (live && g.beta) ld_z<C>(g.Cm, g.ci + mi, g.cj + nj, acr, aci);
  const double asign = g.alpha < 0 ? -1.0 : 1.0;
  for (int64_t k0 = 0; k0 < g.k; k0 += KC) {
    __syncthreads();
    for (int e = t; e < KC * 16; e += 256) {
      const int kk = e % KC, jj = e / KC;
      double re[C], im[C];
      if (k0 + kk < g.k && jj < g.n) {
        if (g.opB == 'N') ld_z<C>(g.B, g.bi + k0 + kk, g.bj + jj, re, im);
        else ld_z<C>(g.B, g.bi + jj, g.bj + k0 + kk, re, im);
        if (g.opB == 'C') {
#pragma unroll
          for (int c = 0; c < C; ++c) im[c] = -im[c];
        }
      } else {
        mp::set_zero<C>(re);
        mp::set_zero<C>(im);
      }
#pragma unroll
      for (int c = 0; c < C; ++c) { sB[kk][0][c][jj] = re[c]; sB[kk][1][c][jj] = im[c]; }
    }
    __syncthreads();
    if (!live) continue;
    const int kend = (g.k - k0 < KC) ? (int)(g.k - k0) : KC;
    for (int kk = 0; kk < kend; ++kk) {
      double ar[C], ai[C], nai[C], br[C], bi[C];
      if (g.opA == 'N') ld_z<C>(g.A, g.ai + mi, g.aj + k0 + kk, ar, ai);
      else ld_z<C>(g.A, g.ai + k0 + kk, g.aj + mi, ar, ai);
      const double isg = (g.opA == 'C') ? -asign : asign;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        ar[c] *= asign;
        ai[c] *= isg;
        nai[c] = -ai[c];
        br[c] = sB[kk][0][c][nj];
        bi[c] = sB[kk][1][c][nj];
      }
      mp::mac<C>(acr, ar, br);
      mp::mac<C>(acr, nai, bi);
      mp::mac<C>(aci, ar, bi);
      mp::mac<C>(aci, ai, br);
      if (g.k > TIDY_MIN_K && ((k0 + kk + 1) % TIDY_K) == 0) {
        mp::tidy<C>(acr);
        mp::tidy<C>(aci);
      }
    }
  }
  if (live) {
    double ore[C], oim[C];
    mp::renorm<C>(acr, ore);
    mp::renorm<C>(aci, oim);
    st_z<C>(g.Cm, g.ci + mi, g.cj + nj, ore, oim);
  }
}

template <int C>
static hipError_t go_narrow(const GemmArgs &a, hipStream_t s) {
  int npow = 1;
  while (npow < a.n) npow <<= 1;
  const int rows_per_block = 256 / npow;
  const int64_t blocks = (a.m + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL((k_gemm_narrow<C>), dim3((unsigned)blocks), dim3(256), 0, s, a, npow);
  return hipGetLastError();
}

template <int C, bool M3, int BM, int BN, int BK, int TM, int TN, int UNR, bool RE = false>
static hipError_t go(const GemmArgs &a, hipStream_t s) {
  constexpr int NT = (BM / TM) * (BN / TN);
  const dim3 grid((unsigned)(((a.n + BN - 1) / BN) * ((a.m + BM - 1) / BM)));
  // double-double 3M and real products of trailing-update depth: cross products on the
  // matrix cores (both tile sizes, so that the tiling never changes a result)
  constexpr bool XMOK = C == 2 && (M3 || RE) && NT == 256 &&
                        ((BM == 32 && BN == 32) || (BM == 16 && BN == 16));
  if (XMOK && a.k <= TIDY_MIN_K)
    hipLaunchKernelGGL((k_gemm<C, M3, BM, BN, BK, TM, TN, UNR, RE, XMOK>), grid, dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_gemm<C, M3, BM, BN, BK, TM, TN, UNR, RE>), grid, dim3(NT), 0, s, a);
  return hipGetLastError();
}

// tile configurations for double-double (index selectable through MPLU_GEMM_CFG while
// tuning); the default, entry 0, unrolls the k loop by two, which lets the level
// accumulators stay in place across iterations instead of being copied at the back edge
template <bool M3>
static hipError_t go_dd(int cfg, const GemmArgs &a, hipStream_t s) {
  switch (cfg) {
    case 1: return go<2, M3, 64, 32, 8, 4, 2, 1>(a, s);
    case 2: return go<2, M3, 64, 64, 8, 4, 4, 1>(a, s);
    case 3: return go<2, M3, 32, 64, 8, 2, 4, 1>(a, s);
    case 4: return go<2, M3, 32, 32, 8, 2, 2, 1>(a, s);
    case 5: return go<2, M3, 64, 32, 8, 4, 2, 2>(a, s);
    case 6: return go<2, M3, 64, 64, 16, 4, 2, 1>(a, s);
    case 7: return go<2, M3, 64, 64, 8, 2, 2, 1>(a, s);
    case 8: return go<2, M3, 32, 32, 16, 2, 2, 2>(a, s);
    default: return go<2, M3, 32, 32, 8, 2, 2, 2>(a, s);
  }
}

static int gemm_cfg() {
  static const int cfg = [] {
    const char *e = getenv("MPLU_GEMM_CFG");
    return e ? atoi(e) : 0;
  }();
  return cfg;
}

hipError_t launch_gemm(int C, int method, char opA, char opB, int64_t m, int64_t n, int64_t k,
                       int alpha_sign, ZM A, int64_t ai, int64_t aj, ZM B, int64_t bi,
                       int64_t bj, int beta, ZM Cm, int64_t ci, int64_t cj, hipStream_t s,
                       bool urgent) {
  if (m <= 0 || n <= 0) return hipSuccess;
  GemmArgs a;
  a.A = A; a.B = B; a.Cm = Cm;
  a.ai = ai; a.aj = aj; a.bi = bi; a.bj = bj; a.ci = ci; a.cj = cj;
  a.m = m; a.n = n; a.k = k;
  a.opA = opA; a.opB = opB;
  a.alpha = alpha_sign; a.beta = beta;
  a.urgent = urgent ? 1 : 0;
  const bool m3 = (method == 1);
  // products too small to give each CU a few 32 x 32 tiles (the next panel's columns in
  // the look-ahead, the last trailing updates) take 16 x 16 tiles, one element per
  // thread; every element still accumulates over k in the same order, so the result does
  // not depend on the tiling
  const bool small = ((m + 31) / 32) * ((n + 31) / 32) < 512;
  if (method == 2) {
    switch (C) {
      case 2: return small ? go<2, false, 16, 16, 16, 1, 1, 2, true>(a, s) : go<2, false, 32, 32, 8, 2, 2, 2, true>(a, s);
      case 3: return small ? go<3, false, 16, 16, 16, 1, 1, 1, true>(a, s) : go<3, false, 32, 32, 8, 2, 2, 1, true>(a, s);
      case 4: return small ? go<4, false, 16, 16, 16, 1, 1, 1, true>(a, s) : go<4, false, 32, 32, 8, 2, 2, 1, true>(a, s);
    }
    return hipErrorInvalidValue;
  }
  if (!m3 && n <= 16) {
    switch (C) {
      case 2: return go_narrow<2>(a, s);
      case 3: return go_narrow<3>(a, s);
      case 4: return go_narrow<4>(a, s);
    }
    return hipErrorInvalidValue;
  }
  switch (C) {
    case 2:
      if (small) return m3 ? go<2, true, 16, 16, 16, 1, 1, 2>(a, s) : go<2, false, 16, 16, 16, 1, 1, 2>(a, s);
      return m3 ? go_dd<true>(gemm_cfg(), a, s) : go_dd<false>(gemm_cfg(), a, s);
    case 3:
      if (small) return m3 ? go<3, true, 16, 16, 16, 1, 1, 1>(a, s) : go<3, false, 16, 16, 16, 1, 1, 1>(a, s);
      return m3 ? go<3, true, 32, 32, 8, 2, 2, 1>(a, s) : go<3, false, 32, 32, 8, 2, 2, 1>(a, s);
    case 4:
      if (small) return m3 ? go<4, true, 16, 16, 16, 1, 1, 1>(a, s) : go<4, false, 16, 16, 16, 1, 1, 1>(a, s);
      return m3 ? go<4, true, 32, 32, 8, 2, 2, 1>(a, s) : go<4, false, 32, 32, 8, 2, 2, 1>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mplu
