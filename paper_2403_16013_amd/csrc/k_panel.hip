// k_panel.hip -- panel factorisation with partial pivoting and the row interchanges it
// implies for the rest of the matrix (Kouya Sec. 3: LU with partial pivoting, blocked
// with panel width K; LAPACK getf2 semantics for the panel).
//
// Design for gfx950: the panel (rows j..m-1, columns j..j+kb-1) is split by rows over G
// co-resident workgroups; each keeps its rows of the panel in LDS for the whole panel.
// Each column costs one grid-wide barrier: before it, every workgroup publishes its local
// pivot candidate (value, row, and the candidate row itself) and the owner of row k
// publishes row k; after it, every workgroup reduces the G candidates to the same winner
// (ties -> lowest row), performs its part of the interchange from the published rows,
// scales its part of the column by the pivot's reciprocal and applies the rank-1 update
// to its rows.  Nothing else touches global memory until the panel is written back.
#include <limits.h>
#include <stdio.h>
#include <stdlib.h>

#include "common.hpp"

#pragma clang fp contract(off)

namespace mplu {

static constexpr int PNT = 256;        // threads per panel workgroup
static constexpr int PGMAX = 256;      // max workgroups (one partial per thread)
static constexpr int PKBMAX = 128;     // max panel width
static constexpr size_t PLDS_BUDGET = 160 * 1024;
static constexpr unsigned SPIN_LIMIT = 1u << 26;  // ~2 s of s_sleep(1) before giving up
static constexpr int32_t MPLU_SYNC_TIMEOUT = -9999;  // mirrors MPLU_INFO_SYNC_TIMEOUT

// ------------------------------------------------------------------ workspace layout
// [0, 256)              barrier words: count, generation, timeout flag
// part  : 2 x (C+1) x PGMAX doubles  (cabs1 components, row index; field-major: field f
//         of workgroup g at f * PGMAX + g)
// rcp   : 2 x 2C x PGMAX doubles  (reciprocal of each candidate pivot, same layout)
// cand  : 2 x PGMAX x 2C x kb doubles
// rowk  : 2 x 2C x kb doubles
// swl   : 1 + 2 x (2 kb) int32  (count, dst rows, src rows)
struct PanelWS {
  unsigned *bar;
  double *part, *rcp, *cand, *rowk;
  int32_t *swl;
};

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static inline PanelWS carve(void *ws, int C, int kb, size_t *total) {
  char *b = (char *)ws;
  size_t off = 256;
  PanelWS w;
  w.bar = (unsigned *)b;
  w.part = (double *)(b + off);
  off = align256(off + sizeof(double) * 2 * PGMAX * (C + 1));
  w.rcp = (double *)(b + off);
  off = align256(off + sizeof(double) * 2 * PGMAX * 2 * C);
  w.cand = (double *)(b + off);
  off = align256(off + sizeof(double) * 2 * PGMAX * 2 * C * kb);
  w.rowk = (double *)(b + off);
  off = align256(off + sizeof(double) * 2 * 2 * C * kb);
  w.swl = (int32_t *)(b + off);
  off = align256(off + sizeof(int32_t) * (1 + 4 * kb));
  if (total) *total = off;
  return w;
}

size_t panel_ws_bytes(int C, int kb) {
  size_t t = 0;
  carve(nullptr, C, kb, &t);
  return t;
}

static inline size_t panel_lds(int C, int kb, int R) {
  const int Q = 2 * C;
  size_t b = sizeof(double) * ((size_t)kb * Q * R + 3 * (size_t)Q * kb + 4 * C + Q);
  b += sizeof(int) * (4 + kb + 4 * kb);
  return align256(b);
}

// compute units of the current device (the panel's workgroups must all be resident)
static int device_cus() {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  int v = cus[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cus[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

PanelGeom panel_geometry(int C, int64_t mp, int kb) {
  PanelGeom g{0, 0, 0};
  if (mp <= 0 || kb <= 0 || kb > PKBMAX) return g;
  // largest row count per workgroup that fits in LDS (and one row per thread)
  int rmax = PNT;
  while (rmax > 1 && panel_lds(C, kb, rmax) > PLDS_BUDGET) --rmax;
  // aim for about 64 workgroups for double-double and 96 for the wider formats: fewer
  // makes the per-column barrier cheaper, more spreads the rank-1 work, whose share grows
  // with the format (measured at n = 4096, panel 64); never below 8 rows each
  // (MPLU_PANEL_WGS and MPLU_PANEL_RMIN override the target and the row floor, for tuning)
  static const int forced = [] {
    const char *e = getenv("MPLU_PANEL_WGS");
    const int t = e ? atoi(e) : 0;
    return t < 1 ? 0 : t;
  }();
  const int target = forced ? forced : (C == 2 ? 64 : 96);
  static const int rmin = [] {
    const char *e = getenv("MPLU_PANEL_RMIN");
    const int t = e ? atoi(e) : 8;
    return t < 1 ? 8 : t;
  }();
  int64_t R = (mp + target - 1) / target;
  if (R < rmin) R = rmin;
  if (R > rmax) R = rmax;
  int64_t G = (mp + R - 1) / R;
  if (G > PGMAX || G > device_cus()) return g;
  g.G = (int)G;
  g.R = (int)R;
  g.lds = panel_lds(C, kb, (int)R);
  return g;
}

struct PanelArgs {
  ZM A;
  int64_t j, m;
  int kb, R, G;
  int32_t *ipiv, *info;
  PanelWS w;
  unsigned base;  // arrival count left by earlier panels on this workspace
};

// lexicographic comparison of renormalised components: a strict total order that
// agrees with the value order of non-overlapping expansions (ties between equal
// representations are broken by the row index)
template <int C>
__device__ __forceinline__ bool better(const double (&a)[C], int ia, const double (&b)[C],
                                       int ib) {
  int c = 0;
#pragma unroll
  for (int k = C - 1; k >= 0; --k) c = (a[k] > b[k]) ? 1 : ((a[k] < b[k]) ? -1 : c);
  // no branches: a missing candidate (row INT_MAX) loses to any present one
  const bool a_ok = ia != INT_MAX, b_ok = ib != INT_MAX;
  return a_ok & (!b_ok | (c > 0) | ((c == 0) & (ia < ib)));
}

// value of lane s of the wave (s uniform across the wave)
__device__ __forceinline__ double lane_value(double v, int s) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), s);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), s);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// a double moved across lanes by the DPP pattern CTRL (within rows of 16 lanes)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int C, int CTRL>
__device__ __forceinline__ void dpp_step(double (&v)[C], int &idx) {
  double ov[C];
#pragma unroll
  for (int c = 0; c < C; ++c) ov[c] = dpp_d<CTRL>(v[c]);
  const int oi = __builtin_amdgcn_update_dpp(0, idx, CTRL, 0xF, 0xF, false);
  if (better<C>(ov, oi, v, idx)) {
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = ov[c];
    idx = oi;
  }
}

// argmax over one wave (all 64 lanes active): rotations by 8, 4, 2, 1 inside each row of
// 16 lanes leave every lane with its row's winner, then the four row winners are read
// out and compared.  "better" is a strict total order on (value, row) pairs, so every
// lane, and every wave reducing the same candidates, ends with the same winner.
template <int C>
__device__ __forceinline__ void wave_argmax(double (&v)[C], int &idx) {
  // Common case first: the largest leading component, by a plain maximum over doubles.
  // When a single lane holds it, that lane's candidate beats every other in the full
  // order, so it is the winner.  Ties on the leading component, and waves whose present
  // candidates are all NaN (the maximum ignores them, and one of them must still win over
  // the missing ones), take the full reduction below; the branches are uniform.
  {
    if (__ballot(idx != INT_MAX) == 0ull) {  // no candidate in the whole wave
#pragma unroll
      for (int c = 0; c < C; ++c) v[c] = 0.0;
      return;
    }
    const double h = (idx == INT_MAX) ? -1.0 : v[0];  // a missing candidate loses
    double m = h;
    m = fmax(m, dpp_d<0x128>(m));
    m = fmax(m, dpp_d<0x124>(m));
    m = fmax(m, dpp_d<0x122>(m));
    m = fmax(m, dpp_d<0x121>(m));
    const double mx = fmax(fmax(lane_value(m, 0), lane_value(m, 16)),
                           fmax(lane_value(m, 32), lane_value(m, 48)));
    const unsigned long long hit = __ballot(h == mx);
    if (mx >= 0.0 && __popcll(hit) == 1) {
      const int s = __ffsll((long long)hit) - 1;
#pragma unroll
      for (int c = 0; c < C; ++c) v[c] = lane_value(v[c], s);
      idx = __builtin_amdgcn_readlane(idx, s);
      return;
    }
  }
  dpp_step<C, 0x128>(v, idx);  // row_ror:8
  dpp_step<C, 0x124>(v, idx);  // row_ror:4
  dpp_step<C, 0x122>(v, idx);  // row_ror:2
  dpp_step<C, 0x121>(v, idx);  // row_ror:1
  double bv[C];
  int bi = __builtin_amdgcn_readlane(idx, 0);
#pragma unroll
  for (int c = 0; c < C; ++c) bv[c] = lane_value(v[c], 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    double ov[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ov[c] = lane_value(v[c], 16 * r);
    const int oi = __builtin_amdgcn_readlane(idx, 16 * r);
    if (better<C>(ov, oi, bv, bi)) {
#pragma unroll
      for (int c = 0; c < C; ++c) bv[c] = ov[c];
      bi = oi;
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) v[c] = bv[c];
  idx = bi;
}

// Cross-workgroup exchange.  Everything one workgroup publishes for the others goes
// through agent-scope atomic stores and is read back with agent-scope atomic loads, which
// are coherent across the XCDs' L2 caches without writing back or invalidating them.  A
// store has reached the coherence point once the issuing wave's memory counter drains,
// so a barrier arrival only needs that wait; no cache-wide fence is used.
__device__ __forceinline__ void put(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double get(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Split grid barrier over G co-resident workgroups: one arrival counter that only grows
// (within a factorisation, consecutive panels sharing a workspace continue from the
// count the previous one left, so it is cleared once per factorisation), polled by the
// waiters.  The wait is bounded and its expiry is sticky (every later wait returns at
// once), so no wave can wait forever.
__device__ __forceinline__ void grid_arrive(unsigned *bar) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's published stores have completed
  __syncthreads();
  // the waiters watch the counter itself, so the old value is not needed
  if (threadIdx.x == 0) __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void grid_wait(unsigned *bar, unsigned want) {
  if (threadIdx.x == 0) {
    unsigned spins = 0;
    while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - want >
           0x7fffffffu) {  // counter < want (modular)
      // the expiry word is looked at only now and then: each look is a round trip
      if ((spins & 255u) == 255u &&
          __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
        break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SPIN_LIMIT) {
        __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}

// A reciprocal slot holds this signalling NaN from the moment its column's barrier is
// entered until the reciprocal is stored.  Arithmetic only ever produces quiet NaNs, so
// a stored reciprocal never has this bit pattern.
static constexpr long long RCP_PENDING = 0x7FF4A5A5A5A5A5A5ll;
__device__ __forceinline__ bool rcp_pending(double v) {
  return __double_as_longlong(v) == RCP_PENDING;
}

// The panel's element operations on complex values, or (RE) on real values: a real
// matrix keeps only its C real planes, the imaginary arrays are then ignored on input and
// returned as zero, the pivot measure is |a| and the reciprocal a real one.
template <int C, bool RE>
__device__ __forceinline__ void pv_cabs1(const double (&re)[C], const double (&im)[C],
                                         double (&o)[C]) {
  if constexpr (RE) mp::abs_<C>(re, o);
  else mp::cabs1<C>(re, im, o);
}

template <int C, bool RE>
__device__ __forceinline__ void pv_recip(const double (&br)[C], const double (&bi)[C],
                                         double (&orr)[C], double (&oi)[C]) {
  if constexpr (RE) {
    mp::recip<C>(br, orr);
    mp::set_zero<C>(oi);
  } else {
    mp::zrecip<C>(br, bi, orr, oi);
  }
}

template <int C, bool RE>
__device__ __forceinline__ void pv_mul(const double (&ar)[C], const double (&ai)[C],
                                       const double (&br)[C], const double (&bi)[C],
                                       double (&orr)[C], double (&oi)[C]) {
  if constexpr (RE) {
    mp::mul<C>(ar, br, orr);
    mp::set_zero<C>(oi);
  } else {
    mp::zmul<C>(ar, ai, br, bi, orr, oi);
  }
}

// o = a - l u, one rounding per part (outputs may alias the inputs)
template <int C, bool RE>
__device__ __forceinline__ void pv_fms(const double (&ar)[C], const double (&ai)[C],
                                       const double (&lr)[C], const double (&li)[C],
                                       const double (&ur)[C], const double (&ui)[C],
                                       double (&orr)[C], double (&oi)[C]) {
  if constexpr (RE) {
    double x[C], nl[C];
    mp::copy<C>(ar, x);
    mp::neg<C>(lr, nl);
    mp::mac<C>(x, nl, ur);
    mp::renorm<C>(x, orr);
    mp::set_zero<C>(oi);
  } else {
    mp::zfms<C>(ar, ai, lr, li, ur, ui, orr, oi);
  }
}

// element (row lr, column c, plane q) of this workgroup's rows in LDS
#define SA(c, q, lr) sA[((size_t)(c) * Q + (q)) * R + (lr)]

// Right-looking panel with look-ahead.  Loop invariant at the top of iteration k: in
// this workgroup's rows, columns <= k are updated through step k-1, columns > k through
// step k-2; the step k-1 update of columns > k ("pending") is applied while the barrier
// of column k is in flight.  Rows published before that update are completed by their
// readers, who hold the previous U row and find the row's multiplier in its column k-1.
template <int C, bool RE>
__global__ __launch_bounds__(PNT) void k_panel(PanelArgs a) {
  extern __shared__ double smem[];
  // the panel is a chain of short dependent steps; when it shares CUs with the trailing
  // update its waves should win instruction issue
  __builtin_amdgcn_s_setprio(3);
  constexpr int Q = RE ? C : 2 * C;  // planes of a value
  constexpr int PREC = C + 1;  // candidate record: cabs1, row
  const int kb = a.kb, R = a.R, G = a.G;
  const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t mp = a.m - a.j;
  const int64_t r0 = (int64_t)g * R;
  const int nr = (int)(mp - r0 < R ? (mp - r0 > 0 ? mp - r0 : 0) : R);
  const ZM A = a.A;
  const int64_t j = a.j;

  double *sA = smem;                             // [kb][Q][R]
  double *sPiv = sA + (size_t)kb * Q * R;        // [Q][kb]  U row k (current pivot row)
  double *sRowK = sPiv + Q * kb;                 // [Q][kb]  row k before the interchange
  double *sPrev = sRowK + Q * kb;                // [Q][kb]  U row k-1
  double *sRedV = sPrev + Q * kb;                // [4][C]
  double *sRcp = sRedV + 4 * C;                  // [Q]
  int *sRedI = (int *)(sRcp + Q);                // [4]
  int *sPivRow = sRedI + 4;                      // [kb]
  int *sList = sPivRow + kb;                     // [4 kb]

  {
    // the panel's rows into LDS: thread t takes row t % nr and every P-th (column, plane)
    // pair from t / nr (P = PNT / nr threads per row), sixteen loads in flight before
    // their stores (one at a time would wait out a memory round trip per element)
    constexpr int LB = 16;
    const int P = nr > 0 ? PNT / nr : 0;
    if (nr > 0 && t < P * nr) {
      const int r = t % nr;
      const double *src = A.p + j + r0 + r;
      for (int cq0 = t / nr; cq0 < kb * Q; cq0 += LB * P) {
        double v[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int cq = cq0 + u * P;  // (column, plane) = (cq / Q, cq % Q)
          if (cq < kb * Q) v[u] = src[(int64_t)(cq % Q) * A.ps + (j + cq / Q) * A.ld];
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int cq = cq0 + u * P;
          if (cq < kb * Q) sA[(size_t)cq * R + r] = v[u];  // SA(cq / Q, cq % Q, r)
        }
      }
    }
  }
  __syncthreads();

  bool prev_zero = true;  // no pending update before column 0
  for (int k = 0; k < kb; ++k) {
    const int par = k & 1;
    double *part = a.w.part + (size_t)par * PGMAX * PREC;
    double *rcpw = a.w.rcp + (size_t)par * PGMAX * Q;
    double *cand = a.w.cand + (size_t)par * PGMAX * Q * kb;
    double *rowk = a.w.rowk + (size_t)par * Q * kb;

    // (1) local pivot candidate among rows >= k (column k is up to date); every wave
    // reduces all of this workgroup's rows, so no workgroup barrier is needed
    double v[C];
    int idx = INT_MAX;
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = 0.0;
    for (int r = lane; r < nr; r += 64) {
      if (r0 + r >= k) {
        double re[C], im[C], cv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          re[c] = SA(k, c, r);
          im[c] = RE ? 0.0 : SA(k, C + c, r);
        }
        pv_cabs1<C, RE>(re, im, cv);
        if (better<C>(cv, (int)(r0 + r), v, idx)) {
#pragma unroll
          for (int c = 0; c < C; ++c) v[c] = cv[c];
          idx = (int)(r0 + r);
        }
      }
    }
    wave_argmax<C>(v, idx);

    // (2) publish the candidate (value, row, row contents) and, if owned, row k
    // (records are stored field by field across workgroups, part[field][g], so that one
    // load instruction of the reader covers 64 workgroups' field in four cache lines)
    if (t == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) put(&part[c * PGMAX + g], v[c]);
      put(&part[C * PGMAX + g], (idx == INT_MAX) ? -1.0 : (double)idx);
      // this slot was last read before the previous column's barrier completed
#pragma unroll
      for (int q = 0; q < Q; ++q) put(&rcpw[q * PGMAX + g], __longlong_as_double(RCP_PENDING));
    }
    if (idx != INT_MAX) {
      const int lr = (int)(idx - r0);
      for (int e = t; e < Q * kb; e += PNT) {
        const int q = e / kb, c = e % kb;
        put(&cand[((size_t)g * Q + q) * kb + c], SA(c, q, lr));
      }
    }
    if (k >= r0 && k < r0 + nr) {
      const int lr = (int)(k - r0);
      for (int e = t; e < Q * kb; e += PNT) {
        const int q = e / kb, c = e % kb;
        put(&rowk[q * kb + c], SA(c, q, lr));
      }
    }
    grid_arrive(a.w.bar);

    // (3) while the barrier is in flight: wave 1 inverts this workgroup's candidate pivot
    // (only the winner's reciprocal will be read, by every workgroup, with the pivot
    // row); waves 0, 2 and 3 apply the pending step k-1 update of columns > k, and for
    // double-double, whose reciprocal is short, wave 1 takes the last eighth of the
    // columns after it (DD 3M gesv 0.3-0.5 ms faster; neutral to slightly slower for TD
    // and QD, where wave 1 stays out)
    if (w == 1 && lane == 0 && idx != INT_MAX) {
      double pr[C], pi[C], rr[C], ri[C];
      const int lr = (int)(idx - r0);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        pr[c] = SA(k, c, lr);
        pi[c] = RE ? 0.0 : SA(k, C + c, lr);
      }
      pv_recip<C, RE>(pr, pi, rr, ri);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        put(&rcpw[c * PGMAX + g], rr[c]);
        if (!RE) put(&rcpw[(C + c) * PGMAX + g], ri[c]);
      }
    }
    if (!prev_zero && k + 1 < kb) {
      const int lo = (int)(k - r0 > 0 ? k - r0 : 0);  // rows with local index >= k
      const int cnt = nr - lo;
      const int ncol = kb - k - 1;
      const int ncol1 = C == 2 ? ncol / 8 : 0;  // wave 1's columns
      const int cb = (w == 1) ? k + 1 + (ncol - ncol1) : k + 1;
      const int nc = (w == 1) ? ncol1 : ncol - ncol1;
      const int tot = cnt * nc;
      const int stride = (w == 1) ? 64 : PNT - 64;
      const int pt = (w == 1) ? lane : ((w == 0) ? t : t - 64);  // index within the group
      // two elements per pass, both loaded before either is computed: their dependent
      // chains of FP64 operations interleave (a lone wave per SIMD otherwise waits out
      // each operation's latency; the wider formats spend most of a column here)
      for (int e = pt; e < tot; e += 2 * stride) {
        const bool two = e + stride < tot;
        const int ee[2] = {e, two ? e + stride : e};
        double xr[2][C], xi[2][C], lr_[2][C], li[2][C], ur[2][C], ui[2][C];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int r = lo + ee[h] % cnt;
          const int c = cb + ee[h] / cnt;
#pragma unroll
          for (int cc = 0; cc < C; ++cc) {
            xr[h][cc] = SA(c, cc, r);
            xi[h][cc] = RE ? 0.0 : SA(c, C + cc, r);
            lr_[h][cc] = SA(k - 1, cc, r);
            li[h][cc] = RE ? 0.0 : SA(k - 1, C + cc, r);
            ur[h][cc] = sPrev[cc * kb + c];
            ui[h][cc] = RE ? 0.0 : sPrev[(C + cc) * kb + c];
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
          pv_fms<C, RE>(xr[h], xi[h], lr_[h], li[h], ur[h], ui[h], xr[h], xi[h]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h == 1 && !two) break;
          const int r = lo + ee[h] % cnt;
          const int c = cb + ee[h] / cnt;
#pragma unroll
          for (int cc = 0; cc < C; ++cc) {
            SA(c, cc, r) = xr[h][cc];
            if (!RE) SA(c, C + cc, r) = xi[h][cc];
          }
        }
      }
    }
    grid_wait(a.w.bar, a.base + (unsigned)G * (unsigned)(k + 1));

    // (4) global winner.  Wave 0 alone loads the G candidate records (one round trip),
    // reduces them, fetches the two rows and, while those are in flight, computes the
    // reciprocal of the pivot, whose complex value came with the winner's record; the
    // other waves pick the results up from LDS.
    if (w == 0) {
      double bv[C];
      int bi = INT_MAX;
#pragma unroll
      for (int c = 0; c < C; ++c) bv[c] = 0.0;
      double pc[PGMAX / 64][C], px[PGMAX / 64];
#pragma unroll
      for (int it = 0; it < PGMAX / 64; ++it) {
        const int gg = lane + 64 * it;
        const bool have = gg < G;
#pragma unroll
        for (int c = 0; c < C; ++c) pc[it][c] = 0.0;
        px[it] = -1.0;
        if (64 * it < G) {  // uniform: slots of absent workgroups are never loaded
#pragma unroll
          for (int c = 0; c < C; ++c) pc[it][c] = have ? get(&part[c * PGMAX + gg]) : 0.0;
          px[it] = have ? get(&part[C * PGMAX + gg]) : -1.0;
        }
      }
#pragma unroll
      for (int it = 0; it < PGMAX / 64; ++it) {
        if (px[it] >= 0.0 && better<C>(pc[it], (int)px[it], bv, bi)) {
#pragma unroll
          for (int c = 0; c < C; ++c) bv[c] = pc[it][c];
          bi = (int)px[it];
        }
      }
      wave_argmax<C>(bv, bi);
      // a winner is always a row >= k of this panel; only records left behind by an
      // expired wait could say otherwise, and they must not steer any address
      if (bi < k || (int64_t)bi >= mp) bi = k;
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) sRedV[c] = bv[c];
        sRedI[0] = bi;
      }
    }
    __syncthreads();
    double bv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) bv[c] = sRedV[c];
    const int p = sRedI[0];
    {
      // every thread fetches its share of the two rows; lanes of wave 1 fetch the
      // winner's reciprocal in the same round trip and wait for it if it is still pending
      const int gp = p / R;
      constexpr int NE = (2 * 4 * PKBMAX + PNT - 1) / PNT;
      double rowv[NE], rowk_v[NE];
      const bool rl = (w == 1) && (lane < Q);
      double rv = rl ? get(&rcpw[lane * PGMAX + gp]) : 0.0;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int e = t + i * PNT;
        if (e < Q * kb) {
          rowv[i] = get(&cand[(size_t)gp * Q * kb + e]);
          rowk_v[i] = get(&rowk[e]);
        }
      }
      if (w == 1) {
        unsigned spins = 0;
        while (__ballot(rl && rcp_pending(rv)) != 0ull) {
          // bounded like the grid barrier, and given up at once after an expiry
          if ((spins & 255u) == 0u &&
              __hip_atomic_load(&a.w.bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            break;
          if (++spins > SPIN_LIMIT) {
            if (lane == 0) __hip_atomic_store(&a.w.bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          if (rl && rcp_pending(rv)) rv = get(&rcpw[lane * PGMAX + gp]);
        }
        if (rl) sRcp[lane] = rv;
      }
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int e = t + i * PNT;
        if (e < Q * kb) {
          sPiv[e] = rowv[i];
          sRowK[e] = rowk_v[i];
        }
      }
    }
    __syncthreads();
    // complete the two published rows with the pending step k-1 update
    if (!prev_zero) {
      for (int e = t; e < 2 * (kb - k - 1); e += PNT) {
        double *row = (e & 1) ? sRowK : sPiv;
        const int c = k + 1 + (e >> 1);
        double xr[C], xi[C], lr_[C], li[C], ur[C], ui[C];
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          xr[cc] = row[cc * kb + c];
          xi[cc] = RE ? 0.0 : row[(C + cc) * kb + c];
          lr_[cc] = row[cc * kb + k - 1];
          li[cc] = RE ? 0.0 : row[(C + cc) * kb + k - 1];
          ur[cc] = sPrev[cc * kb + c];
          ui[cc] = RE ? 0.0 : sPrev[(C + cc) * kb + c];
        }
        pv_fms<C, RE>(xr, xi, lr_, li, ur, ui, xr, xi);
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          row[cc * kb + c] = xr[cc];
          if (!RE) row[(C + cc) * kb + c] = xi[cc];
        }
      }
    }
    bool zero = true;
#pragma unroll
    for (int c = 0; c < C; ++c) zero = zero && (bv[c] == 0.0);
    if (t == 0) {
      sPivRow[k] = p;
      if (g == 0) {
        a.ipiv[j + k] = (int32_t)(j + p + 1);
        if (zero && *a.info == 0) *a.info = (int32_t)(j + k + 1);
      }
    }
    __syncthreads();

    if (!zero) {
      // (5) interchange rows k and p inside this workgroup's rows
      if (p != k) {
        if (p >= r0 && p < r0 + nr) {
          const int lr = (int)(p - r0);
          for (int e = t; e < Q * kb; e += PNT) SA(e % kb, e / kb, lr) = sRowK[e];
        }
        if (k >= r0 && k < r0 + nr) {
          const int lr = (int)(k - r0);
          for (int e = t; e < Q * kb; e += PNT) SA(e % kb, e / kb, lr) = sPiv[e];
        }
      } else if (k >= r0 && k < r0 + nr) {
        const int lr = (int)(k - r0);
        for (int e = t; e < Q * kb; e += PNT) SA(e % kb, e / kb, lr) = sPiv[e];
      }
      __syncthreads();
      // (7) multipliers of column k, then column k+1 brought up to step k
      if (t < nr && r0 + t > k) {
        double xr[C], xi[C], rr[C], ri[C], lr_[C], li[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          xr[c] = SA(k, c, t);
          xi[c] = RE ? 0.0 : SA(k, C + c, t);
          rr[c] = sRcp[c];
          ri[c] = RE ? 0.0 : sRcp[C + c];
        }
        pv_mul<C, RE>(xr, xi, rr, ri, lr_, li);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          SA(k, c, t) = lr_[c];
          if (!RE) SA(k, C + c, t) = li[c];
        }
        if (k + 1 < kb) {
          double ur[C], ui[C];
#pragma unroll
          for (int c = 0; c < C; ++c) {
            xr[c] = SA(k + 1, c, t);
            xi[c] = RE ? 0.0 : SA(k + 1, C + c, t);
            ur[c] = sPiv[c * kb + k + 1];
            ui[c] = RE ? 0.0 : sPiv[(C + c) * kb + k + 1];
          }
          pv_fms<C, RE>(xr, xi, lr_, li, ur, ui, xr, xi);
#pragma unroll
          for (int c = 0; c < C; ++c) {
            SA(k + 1, c, t) = xr[c];
            if (!RE) SA(k + 1, C + c, t) = xi[c];
          }
        }
      }
    }
    // U row k becomes the previous row for the next iteration's pending update
    for (int e = t; e < Q * kb; e += PNT) sPrev[e] = sPiv[e];
    prev_zero = zero;
    __syncthreads();
  }

  {
    // write-back with the load's thread mapping, sixteen LDS reads ahead of their stores
    constexpr int LB = 16;
    const int P = nr > 0 ? PNT / nr : 0;
    if (nr > 0 && t < P * nr) {
      const int r = t % nr;
      double *dst = A.p + j + r0 + r;
      for (int cq0 = t / nr; cq0 < kb * Q; cq0 += LB * P) {
        double v[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int cq = cq0 + u * P;
          if (cq < kb * Q) v[u] = sA[(size_t)cq * R + r];
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int cq = cq0 + u * P;
          if (cq < kb * Q) dst[(int64_t)(cq % Q) * A.ps + (j + cq / Q) * A.ld] = v[u];
        }
      }
    }
  }

  // workgroup 0: the interchange list for the columns outside the panel.  Replaying the
  // kb swaps on the touched rows gives, for every touched row, the row whose content
  // finally lands there (one wave; the search over touched rows uses a ballot).
  if (g == 0 && t < 64) {
    int *rows = sList, *cont = sList + 2 * kb;
    int nt = 0;
    for (int k = 0; k < kb; ++k) {
      const int pr[2] = {k, sPivRow[k]};
      int slot[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        unsigned long long hit = 0;
        for (int base = 0; base < nt; base += 64) {
          const int e = base + t;
          const bool f = (e < nt) && (rows[e] == pr[h]);
          const unsigned long long b = __ballot(f);
          if (b && !hit) hit = ((unsigned long long)(base + __ffsll((long long)b) - 1)) + 1ull;
        }
        if (hit) {
          slot[h] = (int)(hit - 1);
        } else {
          if (t == 0) {
            rows[nt] = pr[h];
            cont[nt] = pr[h];
          }
          slot[h] = nt;
          nt += 1;
        }
        __builtin_amdgcn_wave_barrier();
      }
      if (t == 0 && slot[0] != slot[1]) {
        const int tmp = cont[slot[0]];
        cont[slot[0]] = cont[slot[1]];
        cont[slot[1]] = tmp;
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (t == 0) {
      int cntl = 0;
      int32_t *dst = a.w.swl + 1, *src = a.w.swl + 1 + 2 * kb;
      for (int e = 0; e < nt; ++e)
        if (cont[e] != rows[e]) {
          dst[cntl] = (int32_t)(j + rows[e]);
          src[cntl] = (int32_t)(j + cont[e]);
          ++cntl;
        }
      a.w.swl[0] = cntl;
      if (__hip_atomic_load(&a.w.bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
        *a.info = MPLU_SYNC_TIMEOUT;
    }
  }
}
#undef SA

// RE: a real matrix, C planes
template <int C, bool RE>
__global__ __launch_bounds__(256) void k_laswp(ZM A, int64_t c0, int64_t c1, int64_t n,
                                               const int32_t *swl, int kb) {
  const int cnt = swl[0];
  const int32_t *dst = swl + 1, *src = swl + 1 + 2 * kb;
  const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t ncols = c0 + (n - c1);
  if (w >= ncols) return;
  const int64_t col = w < c0 ? w : c1 + (w - c0);
  constexpr int Q = RE ? C : 2 * C;
  // every read before any write, so the loads of all planes are in flight together; the
  // list (2 kb slots per half) is read in the same round trip as its count
  double *col0 = A.p + col * A.ld;
  double v[4][Q];
  int32_t sr[4], ds[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int e = lane + 64 * h;
    sr[h] = e < 2 * kb ? src[e] : -1;
    ds[h] = e < 2 * kb ? dst[e] : -1;
  }
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const bool live = lane + 64 * h < cnt;
    sr[h] = live ? sr[h] : -1;
    ds[h] = live ? ds[h] : -1;
  }
#pragma unroll
  for (int h = 0; h < 4; ++h)
#pragma unroll
    for (int q = 0; q < Q; ++q) v[h][q] = (sr[h] >= 0) ? col0[(int64_t)q * A.ps + sr[h]] : 0.0;
#pragma unroll
  for (int h = 0; h < 4; ++h)
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (ds[h] >= 0) col0[(int64_t)q * A.ps + ds[h]] = v[h][q];
}

template <int C, bool RE>
static hipError_t launch_panel_t(ZM A, int64_t j, int64_t m, int kb, int32_t *ipiv,
                                 int32_t *info, void *ws, unsigned *base, hipStream_t s) {
  const PanelGeom geo = panel_geometry(C, m - j, kb);
  if (geo.G == 0) return hipErrorInvalidValue;
  PanelArgs a;
  a.A = A;
  a.j = j;
  a.m = m;
  a.kb = kb;
  a.R = geo.R;
  a.G = geo.G;
  a.ipiv = ipiv;
  a.info = info;
  a.w = carve(ws, C, kb, nullptr);
  a.base = *base;
  *base += (unsigned)geo.G * (unsigned)kb;
  static LdsAttr attr;
  const hipError_t ae = attr.ensure((const void *)k_panel<C, RE>, (int)PLDS_BUDGET);
  if (ae != hipSuccess) return ae;
  // G never exceeds the CU count and one workgroup fits a CU, so every workgroup becomes
  // resident once the kernels sharing the device retire theirs: an ordinary launch
  // suffices, and it may run beside the trailing update on another stream.  The real
  // panel uses the complex panel's geometry; its LDS need is at most that.
  hipLaunchKernelGGL((k_panel<C, RE>), dim3(geo.G), dim3(PNT), geo.lds, s, a);
  return hipGetLastError();
}

hipError_t panel_ws_clear(void *ws, bool expire, hipStream_t s) {
  hipError_t e = launch_fill_i32((int32_t *)ws, 0, 4, s);
  if (e != hipSuccess || !expire) return e;
  // the expiry word set before the first wait: every bounded wait gives up at its first
  // look at it and the panel reports MPLU_SYNC_TIMEOUT
  return launch_fill_i32((int32_t *)ws + 2, 1, 1, s);
}

hipError_t launch_panel(int C, ZM A, int64_t j, int64_t m, int kb, int32_t *ipiv,
                        int32_t *info, void *ws, unsigned *base, hipStream_t s, bool real) {
  switch (C) {
    case 2: return real ? launch_panel_t<2, true>(A, j, m, kb, ipiv, info, ws, base, s)
                        : launch_panel_t<2, false>(A, j, m, kb, ipiv, info, ws, base, s);
    case 3: return real ? launch_panel_t<3, true>(A, j, m, kb, ipiv, info, ws, base, s)
                        : launch_panel_t<3, false>(A, j, m, kb, ipiv, info, ws, base, s);
    case 4: return real ? launch_panel_t<4, true>(A, j, m, kb, ipiv, info, ws, base, s)
                        : launch_panel_t<4, false>(A, j, m, kb, ipiv, info, ws, base, s);
  }
  return hipErrorInvalidValue;
}

const int32_t *panel_swap_list(const void *ws, int C, int kb) {
  return carve(const_cast<void *>(ws), C, kb, nullptr).swl;
}

// columns [0, c0) and [c1, n) of A (one wave per column, four per workgroup)
static hipError_t go_laswp(int C, bool real, ZM A, int64_t c0, int64_t c1, int64_t n,
                           const int32_t *swl, int kb, hipStream_t s) {
  const int64_t ncols = c0 + (n - c1);
  if (ncols <= 0) return hipSuccess;
  const dim3 grid((unsigned)((ncols + 3) / 4));
#define LASWP(CC, RR) hipLaunchKernelGGL((k_laswp<CC, RR>), grid, dim3(256), 0, s, A, c0, c1, n, swl, kb)
  switch (C) {
    case 2: if (real) LASWP(2, true); else LASWP(2, false); break;
    case 3: if (real) LASWP(3, true); else LASWP(3, false); break;
    case 4: if (real) LASWP(4, true); else LASWP(4, false); break;
    default: return hipErrorInvalidValue;
  }
#undef LASWP
  return hipGetLastError();
}

hipError_t launch_laswp_list(int C, ZM A, int64_t c0, int64_t ncols, const int32_t *swl,
                             int swstride, hipStream_t s, bool real) {
  if (ncols <= 0) return hipSuccess;
  return go_laswp(C, real, A, 0, c0, c0 + ncols, swl, swstride / 2, s);
}

hipError_t launch_laswp(int C, ZM A, int64_t c0, int64_t c1, int64_t n, const void *ws,
                        int kb, hipStream_t s, bool real) {
  PanelWS w = carve(const_cast<void *>(ws), C, kb, nullptr);
  return go_laswp(C, real, A, c0, c1, n, w.swl, kb, s);
}

}  // namespace mplu
