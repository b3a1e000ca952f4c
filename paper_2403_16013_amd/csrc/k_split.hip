// k_split.hip -- error-free split products on the matrix cores (the Ozaki scheme used by
// Kouya Sec. 2.3 for the multiple-precision matrix product), applied to the 3M complex
// product of Eq. 3m_cemm:  Cm := beta Cm + alpha (T1 - T2) + i alpha (T3 - T1 - T2) with
// T1 = ReX ReY, T2 = ImX ImY, T3 = (ReX + ImX)(ReY + ImY).
//
// Slicing: every vector v of an operand (a row of op(A) or a column of op(B)) gets one
// exponent tau_v with |x| < 2^(tau_v - 1) for all its entries (real part, imaginary part
// and their rounded sum alike), and each entry is written
// as sum_{p=1..S} d_p 2^(tau_v - p W) + (dropped tail) with integer digits
// |d_p| <= 2^(W-1) + 1, taken by round-to-nearest from the multi-component residual.
// Digit products are exact: for INT8 (W = 7) the MFMA accumulates them exactly in INT32;
// for FP64 (W = 22) each level's sum stays below 2^53 for K <= 128 and is exact in FP64.
// All digit-pair products of one level l = p + q <= S + 1 share one accumulator, since
// they carry the same weight 2^(tau_i + tau_j - l W).  The per-level sums are then scaled
// (exact powers of two) and added into multi-component accumulators.
#include <stdlib.h>

#include <type_traits>

#include "common.hpp"

#pragma clang fp contract(off)

namespace mplu {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ slicing
struct SliceArgs {
  ZM M;
  int64_t i0, j0;
  int trans;  // element (v, t) = trans ? M(i0 + t, j0 + v) : M(i0 + v, j0 + t)
  int conj;   // negate the imaginary part
  int neg3;   // negate the digits of the third operand set (Re + Im)
  int64_t nvec, K, Kpad;
  void *out;      // [3][S][nvec][Kpad] digits (int8 or double)
  int32_t *tau;   // [3][nvec]
};

// RE: a real operand; only x[0] (its value) is formed
template <int C, bool RE>
__device__ __forceinline__ void slice_elem(const SliceArgs &a, int64_t v, int64_t t,
                                           double (&x)[3][C]) {
  if (RE) {
    double re[C];
    if (a.trans) ld_re<C>(a.M, a.i0 + t, a.j0 + v, re);
    else ld_re<C>(a.M, a.i0 + v, a.j0 + t, re);
    mp::renorm<C>(re, x[0]);
    return;
  }
  double re[C], im[C];
  if (a.trans) ld_z<C>(a.M, a.i0 + t, a.j0 + v, re, im);
  else ld_z<C>(a.M, a.i0 + v, a.j0 + t, re, im);
  if (a.conj) {
#pragma unroll
    for (int c = 0; c < C; ++c) im[c] = -im[c];
  }
  mp::renorm<C>(re, x[0]);
  mp::renorm<C>(im, x[1]);
  mp::add<C>(x[0], x[1], x[2]);  // the rounded sum of Eq. 3m_cemm
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// one wave per vector; NO operand sets: the three of Eq. 3m_cemm (Re, Im, Re + Im), or
// one for a real operand
template <int C, int W, int S, typename T, int NO>
__global__ __launch_bounds__(256) void k_slice(SliceArgs a) {
  constexpr bool RE = NO == 1;
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= a.nvec) return;
  double mx[3] = {0.0, 0.0, 0.0};
  for (int64_t t = lane; t < a.K; t += 64) {
    double x[3][C];
    slice_elem<C, RE>(a, v, t, x);
#pragma unroll
    for (int o = 0; o < NO; ++o) mx[o] = fmax(mx[o], fabs(x[o][0]));
  }
  // one exponent for the vector's three operand sets (Re, Im, Re + Im): their digits then
  // sit on one grid, so the three level sums of a product carry the same weights and
  // combine exactly in integers (k_split_i8); it bounds each set's entries as well
  double m = 0.0;
#pragma unroll
  for (int o = 0; o < NO; ++o) m = fmax(m, wave_max(mx[o]));
  int e = 0;
  if (m > 0.0) frexp(m, &e);  // m < 2^e, hence every entry (with its tail) < 2^e
  int tau[3];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    tau[o] = m > 0.0 ? e + 1 : 0;
    if (lane == 0) a.tau[o * a.nvec + v] = tau[o];
  }
  T *out = (T *)a.out;
  for (int64_t t = lane; t < a.Kpad; t += 64) {
    double x[3][C];
    if (t < a.K) {
      slice_elem<C, RE>(a, v, t, x);
    } else {
#pragma unroll
      for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int c = 0; c < C; ++c) x[o][c] = 0.0;
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      double r[C];
#pragma unroll
      for (int c = 0; c < C; ++c) r[c] = x[o][c];
#pragma unroll
      for (int p = 1; p <= S; ++p) {
        const double dn = ldexp(1.0, tau[o] - p * W);   // grid
        const double d = rint(ldexp(r[0], p * W - tau[o]));
        r[0] = __builtin_fma(-d, dn, r[0]);  // exact: d*dn is r[0] rounded to the grid
        // bring the residual's leading part back to r[0]
#pragma unroll
        for (int c = C - 1; c > 0; --c) {
          double s, e;
          mp::two_sum(r[c - 1], r[c], s, e);
          r[c - 1] = s;
          r[c] = e;
        }
        // RN digits of -x are those of x negated
        out[(((int64_t)o * S + (p - 1)) * a.nvec + v) * a.Kpad + t] =
            (T)((o == 2 && a.neg3) ? -d : d);
      }
    }
  }
}

// ------------------------------------------------------------------ products
struct SplitArgs {
  const void *xs, *ys;        // digit planes of op(A) (m vectors) and op(B) (n vectors)
  const int32_t *tx, *ty;     // exponents [3][m], [3][n]
  int64_t m, n, Kpad;
  ZM Cm;
  int64_t ci, cj;
  int alpha, beta;
};

// weights of the three real products in the real / imaginary parts
__device__ __forceinline__ void op_signs(int op, double &sr, double &si) {
  sr = (op == 0) ? 1.0 : (op == 1 ? -1.0 : 0.0);
  si = (op == 2) ? 1.0 : -1.0;
}

template <int C, bool RE>
__device__ __forceinline__ void epilogue(const SplitArgs &g, int64_t mi, int64_t nj,
                                         double (&lr)[C], double (&li)[C]) {
  if (mi >= g.m || nj >= g.n) return;
  if (g.alpha < 0) {
#pragma unroll
    for (int c = 0; c < C; ++c) { lr[c] = -lr[c]; li[c] = -li[c]; }
  }
  if (RE) {  // real: only the real planes
    if (g.beta) {
      double cr[C];
      ld_re<C>(g.Cm, g.ci + mi, g.cj + nj, cr);
      mp::push_mp<C>(lr, cr);
    }
    double orr[C];
    mp::renorm<C>(lr, orr);
    st_re<C>(g.Cm, g.ci + mi, g.cj + nj, orr);
    return;
  }
  if (g.beta) {
    double cr[C], cim[C];
    ld_z<C>(g.Cm, g.ci + mi, g.cj + nj, cr, cim);
    mp::push_mp<C>(lr, cr);
    mp::push_mp<C>(li, cim);
  }
  double orr[C], oi[C];
  mp::renorm<C>(lr, orr);
  mp::renorm<C>(li, oi);
  st_z<C>(g.Cm, g.ci + mi, g.cj + nj, orr, oi);
}

typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

// rows i .. i+3 of column j in each of the NQ planes of M, the first nv of them (a lane of
// a 16 x 16 MFMA block holds four consecutive rows of one column): two 16-byte loads per
// plane when all four are inside, else one element at a time; absent rows read as zero
template <int NQ>
__device__ __forceinline__ void ld_col4(const ZM &M, int64_t i, int64_t j, int nv,
                                        double (&v)[NQ][4]) {
  const double *b = M.p + j * M.ld + i;
  if (nv == 4) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const d2u lo = *(const d2u *)(b + (int64_t)q * M.ps);
      const d2u hi = *(const d2u *)(b + (int64_t)q * M.ps + 2);
      v[q][0] = lo.x; v[q][1] = lo.y; v[q][2] = hi.x; v[q][3] = hi.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) v[q][e] = e < nv ? b[(int64_t)q * M.ps + e] : 0.0;
  }
}

template <int NQ>
__device__ __forceinline__ void st_col4(const ZM &M, int64_t i, int64_t j, int nv,
                                        const double (&v)[NQ][4]) {
  double *b = M.p + j * M.ld + i;
  if (nv == 4) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      *(d2u *)(b + (int64_t)q * M.ps) = d2u{v[q][0], v[q][1]};
      *(d2u *)(b + (int64_t)q * M.ps + 2) = d2u{v[q][2], v[q][3]};
    }
  } else {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (e < nv) b[(int64_t)q * M.ps + e] = v[q][e];
  }
}

// epilogue of the four outputs (rows i .. i+3 of column j) of one lane, with the values
// of C they update already in registers (cv, planes of the real then the imaginary part)
template <int C, bool RE>
__device__ __forceinline__ void epilogue4(const SplitArgs &g, int64_t i, int64_t j, int nv,
                                          double (&lr)[4][C], double (&li)[4][C],
                                          const double (&cv)[RE ? C : 2 * C][4]) {
  if (nv == 0) return;
  constexpr int NQ = RE ? C : 2 * C;
  double out[NQ][4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (g.alpha < 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) { lr[e][c] = -lr[e][c]; li[e][c] = -li[e][c]; }
    }
    if (g.beta) {
      double cr[C];
#pragma unroll
      for (int c = 0; c < C; ++c) cr[c] = cv[c][e];
      mp::push_mp<C>(lr[e], cr);
      if (!RE) {
        double cim[C];
#pragma unroll
        for (int c = 0; c < C; ++c) cim[c] = cv[(RE ? 0 : C) + c][e];
        mp::push_mp<C>(li[e], cim);
      }
    }
    double o[C];
    mp::renorm<C>(lr[e], o);
#pragma unroll
    for (int c = 0; c < C; ++c) out[c][e] = o[c];
    if (!RE) {
      mp::renorm<C>(li[e], o);
#pragma unroll
      for (int c = 0; c < C; ++c) out[(RE ? 0 : C) + c][e] = o[c];
    }
  }
  st_col4<NQ>(g.Cm, g.ci + i, g.cj + j, nv, out);
}

// INT8 digits, W = 7.  Workgroup: 4 waves, a 32 x 32 output tile; each wave a 16 x 16
// block.  For each real product and each 64-deep k chunk the workgroup stages the S digit
// planes of its 32 rows and 32 columns in LDS (16 bytes per lane, shared by the four
// waves); each wave then holds the S row fragments and S column fragments of its block in
// registers and issues one MFMA per digit pair p + q <= S - 1 (0-based) into the level
// accumulator of that pair: all pairs of one level share it.
//
// The planes are loaded straight into LDS (global-to-LDS, one 16-byte piece per lane at
// the wave's base + 16 x lane).  With one staging buffer per workgroup two workgroups
// share a CU (for double-double), so one's MFMAs run while the other waits for its planes
// or flushes its levels; this measured faster than a second buffer per workgroup.  Rows
// and columns past the edge load the last valid one: they only reach outputs that are
// never stored.  (A permutation of each row's four 16-byte quarters in LDS, spreading a
// fragment read's 16 rows over distinct banks, measured no faster and left the
// bank-conflict counter unchanged.)
template <int C, int S, int NO>
__global__ __launch_bounds__(256) void k_split_i8(SplitArgs g) {
  constexpr int W = 7;
  constexpr bool RE = NO == 1;
  constexpr int PL = S * 32 * 4;            // 16-byte pieces per operand per chunk
  extern __shared__ v4i sdig[];             // [2][S][32 rows][4 x 16 bytes]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t tm, tn;
  xcd_tile((g.m + 31) / 32, (g.n + 31) / 32, tm, tn);
  const int64_t M0 = tm * 32, N0 = tn * 32;
  const int64_t m0 = M0 + 16 * (w >> 1), n0 = N0 + 16 * (w & 1);
  const int64_t bcol = n0 + (lane & 15);
  const int frow = 16 * (w >> 1) + (lane & 15), fcol = 16 * (w & 1) + (lane & 15);
  const int fk = lane >> 4;   // which 16-byte quarter of the 64-deep chunk
  // LDS slots of this lane's quarter of its fragment row and column
  const int xslot = frow * 4 + fk, yslot = fcol * 4 + fk;
  const int8_t *xs = (const int8_t *)g.xs, *ys = (const int8_t *)g.ys;
  double lr[4][C], li[4][C];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int c = 0; c < C; ++c) { lr[e][c] = 0.0; li[e][c] = 0.0; }

  // the exponent sums of this lane's four outputs for the three products, fetched up
  // front so the per-product flush does not wait on memory
  // (one exponent per row / column serves all three products)
  int tsums[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t mi = m0 + 4 * (lane >> 4) + e, nj = bcol;
    tsums[e] = (mi < g.m ? g.tx[mi] : 0) + (nj < g.n ? g.ty[nj] : 0);
  }
  // the values of C this lane's outputs update, fetched now so that their latency
  // overlaps the products
  const int64_t rb = m0 + 4 * (lane >> 4);
  const int nv = (bcol < g.n && rb < g.m) ? (int)(g.m - rb < 4 ? g.m - rb : 4) : 0;
  double cv[RE ? C : 2 * C][4];
  ld_col4<RE ? C : 2 * C>(g.Cm, g.ci + rb, g.cj + bcol, g.beta ? nv : 0, cv);
  const int nck = (int)(g.Kpad / 64);
  // The fill: piece e = (plane p, row r, quarter f) of a chunk goes to slot e of the
  // staging buffer.  Wave w fills the pieces w * 64 + 256 i + lane: planes 2 i + w / 2,
  // rows 16 (w & 1) + lane / 4, quarter lane & 3, so each lane's source row and quarter
  // are the same in every plane and chunk.
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const int8_t *px, *py;
  {
    const int r = 16 * (wu & 1) + (lane >> 2);
    const int f = lane & 3;
    const int64_t gi = (M0 + r < g.m) ? M0 + r : g.m - 1;
    const int64_t gj = (N0 + r < g.n) ? N0 + r : g.n - 1;
    px = xs + gi * g.Kpad + 16 * f;
    py = ys + gj * g.Kpad + 16 * f;
  }
  const int64_t psx = g.m * g.Kpad, psy = g.n * g.Kpad;  // plane strides
  // chunk `it` (product it / nck)
  auto issue = [&](int it) {
    const int op = it / nck;
    const int64_t kc = (int64_t)(it - op * nck) * 64;
    const int pl0 = op * S + (wu >> 1);
    const int8_t *qx = px + pl0 * psx + kc, *qy = py + pl0 * psy + kc;
    v4i *dX = sdig, *dY = sdig + PL;
#pragma unroll
    for (int i = 0; i < (S + 1) / 2; ++i) {
      if (2 * i + (wu >> 1) < S) {
        const int e0 = wu * 64 + 256 * i;
        __builtin_amdgcn_global_load_lds((const void *)qx,
                                         (__attribute__((address_space(3))) void *)(dX + e0),
                                         16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)qy,
                                         (__attribute__((address_space(3))) void *)(dY + e0),
                                         16, 0, 0);
      }
      qx += 2 * psx;
      qy += 2 * psy;
    }
  };
  // Level l (0-based) of a product carries weight 2^(tau_i + tau_j - (l + 2) W), the same
  // for the three products of Eq. 3m_cemm (one exponent per row / column for all three),
  // so they combine exactly in INT32 in one set of level accumulators.  The digits of the
  // third operand set of op(A) arrive negated, so the accumulators hold T1, then T1 + T2,
  // then T1 + T2 - T3: twice the first goes to the real part, the second is subtracted
  // from it (leaving T1 - T2) and the third is subtracted from the imaginary part
  // (leaving T3 - T1 - T2).  Three flushes instead of five.
  // Four consecutive levels span at most 26 + 3 W bits (|sum| < 3 x 64 S 65^2 per chunk,
  // below 2^31 by the depth limit), so their scaled sum is exact in binary64.  A group
  // starting at level lo is at most 2^(-lo W) of the largest possible level-0 sum, so it
  // enters the accumulator at component level lo W / 53: the TwoSum steps above that
  // level would only pass it down unchanged.
  // The levels of a finished product are copied out of the accumulators and pushed into
  // the multi-component sums while the next product's first chunk is in flight.
  v4i acc[S], snap[S];
#pragma unroll
  for (int l = 0; l < S; ++l) acc[l] = v4i{0, 0, 0, 0};
  auto chunk = [&]() {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's pieces of the chunk have landed
    __syncthreads();                // and everybody else's
    const v4i *sX = sdig, *sY = sdig + PL;
    v4i a[S], b[S];
#pragma unroll
    for (int p = 0; p < S; ++p) {
      a[p] = sX[p * 128 + xslot];
      b[p] = sY[p * 128 + yslot];
    }
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S - p; ++q)
        acc[p + q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[p], b[q], acc[p + q], 0, 0, 0);
    __syncthreads();  // the buffer is refilled next
  };
  // product op: its levels scaled by 2 and added (op 0), or subtracted (ops 1 and 2); op 2
  // goes to the imaginary part.  A real product (one operand set) adds its levels to the
  // real part.
  auto flush = [&](int op) {
    const int sc = (!RE && op == 0) ? 1 : 0;  // power of two
    const bool to_re = RE || op < 2;
    const bool sub = !RE && op > 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int tsum = tsums[e] + sc;
#pragma unroll
      for (int top = S - 1; top >= 0; top -= 4) {
        const int lo = top - 3 < 0 ? 0 : top - 3;
        const int lvl = (lo * W) / 53 < C - 1 ? (lo * W) / 53 : C - 1;
        double grp = 0.0;
#pragma unroll
        for (int l = top; l >= lo; --l)
          grp = __builtin_fma((double)snap[l][e], ldexp(1.0, (lo - l) * W), grp);
        grp = ldexp(sub ? -grp : grp, tsum - (lo + 2) * W);
        if (to_re) mp::push<C>(lr[e], lvl, grp);
        else mp::push<C>(li[e], lvl, grp);
      }
    }
  };
  for (int op = 0; op < NO; ++op) {
    issue(op * nck);
    if (op > 0) flush(op - 1);
    chunk();
    for (int c = 1; c < nck; ++c) {
      issue(op * nck + c);
      chunk();
    }
    // the copy lives in VGPRs; without the opaque step the compiler would keep reading
    // the old accumulators and give the next product a second set (twice the registers)
#pragma unroll
    for (int l = 0; l < S; ++l) {
      snap[l] = acc[l];
      asm volatile("" : "+v"(snap[l]));
    }
  }
  flush(NO - 1);
  epilogue4<C, RE>(g, rb, bcol, nv, lr, li, cv);
}

// FP64 digits, W = 22, K processed in blocks of 128 (the exactness limit of one level).
// D layout of the 16x16x4 FP64 MFMA: element (4 e + lane/16, lane % 16) in register e.
// The digits are staged in LDS: the four waves of a workgroup share each 16-deep chunk of
// the digit planes of their 32 rows and 32 columns (loaded straight from memory, every
// fragment was fetched by two waves and the fetches held the MFMAs back).  Piece e (16
// bytes: two consecutive k) of a plane's chunk goes to LDS slot e, which is element
// (step s, row r, k 4 s + kk) at ((s * 32 + r) * 4 + kk): a fragment read (16 rows x 4 k
// of one step) is 64 consecutive doubles.
//   DD: the pieces go straight to LDS (48 KB for S = 6); two workgroups share a CU, so
//       one's MFMAs run while the other's chunk loads.
//   TD, QD (72 and 88 KB, one workgroup per CU): the next chunk's pieces are loaded into
//       registers while this chunk's MFMAs run and written to LDS after them.
template <int C, int S, int NO>
__global__ __launch_bounds__(256, C == 2 ? 2 : 1) void k_split_f64_lds(SplitArgs g) {
  constexpr int W = 22, KC = 16, PL = 32 * KC / 2;  // 16-byte pieces per plane per chunk
  constexpr bool RE = NO == 1, DMA = C == 2;
  typedef double v2d __attribute__((ext_vector_type(2)));
  extern __shared__ double sfd[];  // [2 operands][S planes][PL pieces of 2 doubles]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t M0 = (int64_t)blockIdx.y * 32, N0 = (int64_t)blockIdx.x * 32;
  const int64_t m0 = M0 + 16 * (w >> 1), n0 = N0 + 16 * (w & 1);
  const int64_t bcol = n0 + (lane & 15);
  const int kl = lane >> 4;
  const int rA = 16 * (w >> 1) + (lane & 15), rB = 16 * (w & 1) + (lane & 15);
  const double *xs = (const double *)g.xs, *ys = (const double *)g.ys;
  const int wu = __builtin_amdgcn_readfirstlane(w);
  // the piece this thread fetches in every plane and chunk: step t / 64, row (t / 2) % 32,
  // k pair 2 (t % 2); rows and columns past the edge fetch the last valid one (they only
  // reach outputs that are never stored)
  const int fs = t >> 6, fr = (t >> 1) & 31, fk = 2 * (t & 1);
  const int64_t gi = (M0 + fr < g.m) ? M0 + fr : g.m - 1;
  const int64_t gj = (N0 + fr < g.n) ? N0 + fr : g.n - 1;
  const double *px = xs + gi * g.Kpad + 4 * fs + fk;
  const double *py = ys + gj * g.Kpad + 4 * fs + fk;
  const int64_t psx = g.m * g.Kpad, psy = g.n * g.Kpad;  // plane strides
  v2d rx[S], ry[S];  // register staging (TD, QD)
  auto fetch = [&](int op, int64_t kc) {
#pragma unroll
    for (int p = 0; p < S; ++p) {
      if (DMA) {
        __builtin_amdgcn_global_load_lds(
            (const void *)(px + ((int64_t)op * S + p) * psx + kc),
            (__attribute__((address_space(3))) void *)(sfd + ((size_t)p * PL + wu * 64) * 2), 16,
            0, 0);
        __builtin_amdgcn_global_load_lds(
            (const void *)(py + ((int64_t)op * S + p) * psy + kc),
            (__attribute__((address_space(3))) void *)(sfd + ((size_t)(S + p) * PL + wu * 64) * 2),
            16, 0, 0);
      } else {
        rx[p] = *(const v2d *)(px + ((int64_t)op * S + p) * psx + kc);
        ry[p] = *(const v2d *)(py + ((int64_t)op * S + p) * psy + kc);
      }
    }
  };
  auto store = [&]() {  // register staging into LDS
#pragma unroll
    for (int p = 0; p < S; ++p) {
      *(v2d *)(sfd + ((size_t)p * PL + t) * 2) = rx[p];
      *(v2d *)(sfd + ((size_t)(S + p) * PL + t) * 2) = ry[p];
    }
  };
  double lr[4][C], li[4][C];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) { lr[q][c] = 0.0; li[q][c] = 0.0; }

  if (!DMA) fetch(0, 0);
  for (int op = 0; op < NO; ++op) {
    double sr, si;
    op_signs(op, sr, si);
    if (RE) si = 0.0;
    for (int64_t kb = 0; kb < g.Kpad; kb += 128) {
      const int64_t kend = (kb + 128 < g.Kpad) ? kb + 128 : g.Kpad;
      v4d acc[S];
#pragma unroll
      for (int l = 0; l < S; ++l) acc[l] = v4d{0.0, 0.0, 0.0, 0.0};
      if (DMA) fetch(op, kb);
      for (int64_t kc = kb; kc < kend; kc += KC) {
        if (DMA) {
          __builtin_amdgcn_s_waitcnt(0);  // this wave's pieces have landed
        } else {
          store();
          // the next chunk (of this block, else of the next block or product) is fetched
          // into the registers while this one is multiplied
          int64_t nk = kc + KC;
          int nop = op;
          if (nk >= kend) {
            nk = kend;
            if (nk >= g.Kpad) { nk = 0; ++nop; }
          }
          if (nop < NO) fetch(nop, nk);
        }
        __syncthreads();  // every wave's pieces are in LDS
#pragma unroll
        for (int st = 0; st < KC / 4; ++st) {
          double a[S], b[S];
#pragma unroll
          for (int p = 0; p < S; ++p) {
            a[p] = sfd[(size_t)p * PL * 2 + (st * 32 + rA) * 4 + kl];
            b[p] = sfd[(size_t)(S + p) * PL * 2 + (st * 32 + rB) * 4 + kl];
          }
#pragma unroll
          for (int p = 0; p < S; ++p)
#pragma unroll
            for (int q = 0; q < S - p; ++q)
              acc[p + q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p + q], 0, 0, 0);
        }
        __syncthreads();  // the buffer is refilled next
        if (DMA && kc + KC < kend) fetch(op, kc + KC);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t mi = m0 + 4 * q + (lane >> 4), nj = bcol;
        const int tsum = (mi < g.m ? g.tx[(int64_t)op * g.m + mi] : 0) +
                         (nj < g.n ? g.ty[(int64_t)op * g.n + nj] : 0);
#pragma unroll
        for (int l = S - 1; l >= 0; --l) {
          const int lvl = (l * W) / 53 < C - 1 ? (l * W) / 53 : C - 1;
          const double v = ldexp(acc[l][q], tsum - (l + 2) * W);
          if (sr != 0.0) mp::push<C>(lr[q], lvl, sr * v);
          if (!RE) mp::push<C>(li[q], lvl, si * v);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) epilogue<C, RE>(g, m0 + 4 * q + (lane >> 4), bcol, lr[q], li[q]);
}

// ------------------------------------------------------------------ host side
static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int split_slices(int C, bool i8) {
  if (i8) return C == 2 ? 17 : (C == 3 ? 24 : 32);
  return C == 2 ? 6 : (C == 3 ? 9 : 11);
}

static inline int64_t kpad_of(int64_t K, bool i8) {
  const int64_t q = i8 ? 64 : 16;  // the INT8 chunk, the FP64 double-double chunk
  return ((K + q - 1) / q) * q;
}

// Depth of one INT8 split product.  A level sum of k_split_i8 gains at most 64 S 65^2 per
// 64-deep chunk (S digit pairs of at most 65 x 65 at the top level), and the combined
// sums of the complex product (T1 - T2, T3 - T1 - T2) up to three times that, so they stay
// below 2^31 for floor((2^31 - 1) / (3 x 64 S 65^2)) chunks: 155 (DD), 110 (TD), 82 (QD),
// i.e. k up to 9 920, 7 040, 5 248.
static int64_t split_i8_max_k(int S) { return (2147483647ll / (3ll * 64 * S * 65 * 65)) * 64; }

size_t split_ws_bytes(int C, bool i8, int64_t m, int64_t n, int64_t K, int S) {
  if (S <= 0) S = split_slices(C, i8);
  if (i8 && K > split_i8_max_k(S)) K = split_i8_max_k(S);  // deeper products run in pieces
  const size_t el = i8 ? 1 : 8;
  const int64_t Kp = kpad_of(K, i8);
  size_t b = al256(el * 3 * (size_t)S * (size_t)m * (size_t)Kp);
  b += al256(el * 3 * (size_t)S * (size_t)n * (size_t)Kp);
  b += al256(sizeof(int32_t) * 3 * (size_t)m) + al256(sizeof(int32_t) * 3 * (size_t)n);
  return b;
}

// NO = 3 operand sets (complex, Eq. 3m_cemm) or 1 (real); the workspace layout is the
// complex one in both cases
template <int C, int S, bool I8, int NO>
static hipError_t run(char opA, char opB, int64_t m, int64_t n, int64_t k, int alpha, ZM A,
                      int64_t ai, int64_t aj, ZM B, int64_t bi, int64_t bj, int beta, ZM Cm,
                      int64_t ci, int64_t cj, void *ws, hipStream_t s) {
  typedef typename std::conditional<I8, int8_t, double>::type T;
  constexpr int W = I8 ? 7 : 22;
  const int64_t Kp = kpad_of(k, I8);
  char *p = (char *)ws;
  SliceArgs sx, sy;
  sx.M = A; sx.i0 = ai; sx.j0 = aj; sx.trans = (opA != 'N'); sx.conj = (opA == 'C');
  sx.neg3 = I8 && NO == 3;  // k_split_i8 forms -T3 (see there)
  sx.nvec = m; sx.K = k; sx.Kpad = Kp;
  sx.out = p;
  p += al256(sizeof(T) * 3 * (size_t)S * (size_t)m * (size_t)Kp);
  sy.M = B; sy.i0 = bi; sy.j0 = bj; sy.trans = (opB == 'N'); sy.conj = (opB == 'C');
  sy.neg3 = 0;
  sy.nvec = n; sy.K = k; sy.Kpad = Kp;
  sy.out = p;
  p += al256(sizeof(T) * 3 * (size_t)S * (size_t)n * (size_t)Kp);
  sx.tau = (int32_t *)p;
  p += al256(sizeof(int32_t) * 3 * (size_t)m);
  sy.tau = (int32_t *)p;
  hipLaunchKernelGGL((k_slice<C, W, S, T, NO>), dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, sx);
  hipLaunchKernelGGL((k_slice<C, W, S, T, NO>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, sy);
  SplitArgs g;
  g.xs = sx.out; g.ys = sy.out; g.tx = sx.tau; g.ty = sy.tau;
  g.m = m; g.n = n; g.Kpad = Kp;
  g.Cm = Cm; g.ci = ci; g.cj = cj; g.alpha = alpha; g.beta = beta;
  const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
  if constexpr (I8) {
    const dim3 grid1((unsigned)(((n + 31) / 32) * ((m + 31) / 32)));
    const size_t lds = sizeof(v4i) * 2 * S * 32 * 4;
    static LdsAttr attr;
    const hipError_t e = attr.ensure((const void *)k_split_i8<C, S, NO>, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_split_i8<C, S, NO>), grid1, dim3(256), lds, s, g);
  } else {
    const size_t lds = sizeof(double) * 2 * 2 * S * (32 * 16 / 2);
    static LdsAttr attr;
    const hipError_t e = attr.ensure((const void *)k_split_f64_lds<C, S, NO>, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_split_f64_lds<C, S, NO>), grid, dim3(256), lds, s, g);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_split(int C, bool i8, int S, char opA, char opB, int64_t m, int64_t n,
                             int64_t k, int alpha, ZM A, int64_t ai, int64_t aj, ZM B,
                             int64_t bi, int64_t bj, int beta, ZM Cm, int64_t ci, int64_t cj,
                             void *ws, hipStream_t s, bool real) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (S <= 0) S = split_slices(C, i8);
  if (i8 && k > split_i8_max_k(S)) {
    // deeper products run as consecutive pieces accumulated into Cm (beta = 1 after the
    // first); each piece adds one rounding of the running sum
    const int64_t kp = split_i8_max_k(S);
    for (int64_t k0 = 0; k0 < k; k0 += kp) {
      const int64_t kk = k - k0 < kp ? k - k0 : kp;
      const bool ta = opA != 'N', tb = opB != 'N';
      const hipError_t e = launch_gemm_split(
          C, i8, S, opA, opB, m, n, kk, alpha, A, ai + (ta ? k0 : 0), aj + (ta ? 0 : k0), B,
          bi + (tb ? 0 : k0), bj + (tb ? k0 : 0), k0 == 0 ? beta : 1, Cm, ci, cj, ws, s, real);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
#define RUN(CC, SS, II)                                                                      \
  return real ? run<CC, SS, II, 1>(opA, opB, m, n, k, alpha, A, ai, aj, B, bi, bj, beta, Cm, ci, cj, ws, s) \
              : run<CC, SS, II, 3>(opA, opB, m, n, k, alpha, A, ai, aj, B, bi, bj, beta, Cm, ci, cj, ws, s)
  if (i8) {
    if (C == 2 && S == 17) RUN(2, 17, true);
    if (C == 3 && S == 24) RUN(3, 24, true);
    if (C == 4 && S == 32) RUN(4, 32, true);
  } else {
    if (C == 2) {
      if (S == 3) RUN(2, 3, false);
      if (S == 4) RUN(2, 4, false);
      if (S == 5) RUN(2, 5, false);
      if (S == 6) RUN(2, 6, false);
    }
    if (C == 3 && S == 9) RUN(3, 9, false);
    if (C == 4 && S == 11) RUN(4, 11, false);
  }
#undef RUN
  return hipErrorInvalidValue;
}

bool split_supported(int C, bool i8, int S) {
  if (S <= 0) return true;
  if (i8) return S == split_slices(C, true);
  if (C == 2) return S >= 3 && S <= 6;
  return S == split_slices(C, false);
}

}  // namespace mplu
