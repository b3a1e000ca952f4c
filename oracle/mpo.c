/*
 * mpo.c -- plain, slow, exact-then-round CPU reference for complex multi-component
 * LU with partial pivoting (double-double, triple-double, quadruple-double).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls this
 * file: only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * do.  It shares no code, header, table or helper with the GPU library.
 *
 * Number format (Kouya, Sec. 1 and Sec. 2.2, Fig. 1): a real multiple-precision value
 * is an unevaluated sum of C binary64 components, C = 2 (DD, 106 bits), 3 (TD, 159 bits)
 * or 4 (QD, 212 bits).  A complex matrix keeps real and imaginary parts in separate
 * arrays.  Here a matrix is 2*C planes: plane q = ri*C + c (ri = 0 real, 1 imaginary) at
 * base + q*ps, each plane column-major with leading dimension ld.
 *
 * Rounding rule for EVERY operation in this file: the exact result is formed as a big
 * binary integer, then rounded greedily, c0 = RN(x), c1 = RN(x - c0), c2 = RN(x - c0 - c1),
 * ... (RN = round to nearest, ties to even).  The result is canonical and unique, so a
 * test can recompute it bit for bit with exact rational arithmetic.  Components that
 * would fall below 2^-1022 are flushed to zero (never reached by the workloads here).
 *
 * Threading: OpenMP only splits independent output elements (rows of an update, right-
 * hand sides, rows of a product).  Every element sees the same operation sequence for
 * any thread count, so results are bitwise independent of the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------------------ */
/* Exact fixed-point magnitudes: value = sum_i w[i] * 2^(64 i + XBASE).                   */
/* Only limbs lo..hi are meaningful; the others are treated as zero.                     */
/* XBASE is below the lowest bit of any product of two doubles (2^-2252), and XW limbs    */
/* reach above 2^2300, beyond any product of two finite doubles plus carries.             */
/* ------------------------------------------------------------------------------------ */
#define XW 72
#define XBASE (-2304)

typedef struct {
  uint64_t w[XW];
  int lo, hi;
} xmag;

static inline void xm_clear(xmag *x) { x->lo = 0; x->hi = -1; }
static inline int xm_empty(const xmag *x) { return x->hi < x->lo; }
static inline uint64_t xm_get(const xmag *x, int i) {
  return (i >= x->lo && i <= x->hi) ? x->w[i] : 0;
}

static inline void xm_touch(xmag *x, int a, int b) {
  if (b >= XW) b = XW - 1;
  if (a < 0) a = 0;
  if (xm_empty(x)) {
    for (int i = a; i <= b; i++) x->w[i] = 0;
    x->lo = a;
    x->hi = b;
    return;
  }
  if (a < x->lo) {
    for (int i = a; i < x->lo; i++) x->w[i] = 0;
    x->lo = a;
  }
  if (b > x->hi) {
    for (int i = x->hi + 1; i <= b; i++) x->w[i] = 0;
    x->hi = b;
  }
}

static inline void xm_trim(xmag *x) {
  while (x->hi >= x->lo && x->w[x->hi] == 0) x->hi--;
  while (x->lo <= x->hi && x->w[x->lo] == 0) x->lo++;
  if (x->hi < x->lo) xm_clear(x);
}

/* x += m * 2^p (p >= 0 counted from XBASE) */
static inline void xm_add_at(xmag *x, u128 m, int p) {
  int li = p >> 6, sh = p & 63;
  uint64_t m0 = (uint64_t)m, m1 = (uint64_t)(m >> 64);
  uint64_t t0 = m0 << sh;
  uint64_t t1 = sh ? ((m1 << sh) | (m0 >> (64 - sh))) : m1;
  uint64_t t2 = sh ? (m1 >> (64 - sh)) : 0;
  xm_touch(x, li, li + 2);
  u128 s = (u128)x->w[li] + t0;
  x->w[li] = (uint64_t)s;
  s = (u128)x->w[li + 1] + t1 + (uint64_t)(s >> 64);
  x->w[li + 1] = (uint64_t)s;
  s = (u128)x->w[li + 2] + t2 + (uint64_t)(s >> 64);
  x->w[li + 2] = (uint64_t)s;
  uint64_t c = (uint64_t)(s >> 64);
  for (int i = li + 3; c && i < XW; i++) {
    xm_touch(x, i, i);
    x->w[i] += 1;
    c = (x->w[i] == 0);
  }
}

static int xm_msb(const xmag *x) {
  for (int i = x->hi; i >= x->lo; i--)
    if (x->w[i]) return 64 * i + 63 - __builtin_clzll(x->w[i]);
  return -1;
}

static inline int xm_bit(const xmag *x, int b) {
  if (b < 0) return 0;
  return (int)((xm_get(x, b >> 6) >> (b & 63)) & 1u);
}

/* cnt (<= 64) bits starting at bit position low >= 0 */
static inline uint64_t xm_bits(const xmag *x, int low, int cnt) {
  int li = low >> 6, sh = low & 63;
  u128 v = ((u128)xm_get(x, li + 1) << 64) | xm_get(x, li);
  uint64_t r = (uint64_t)(v >> sh);
  return cnt >= 64 ? r : (r & ((1ULL << cnt) - 1));
}

/* any bit set strictly below position b */
static int xm_any_below(const xmag *x, int b) {
  if (b <= 0) return 0;
  int li = b >> 6;
  for (int i = x->lo; i < li && i <= x->hi; i++)
    if (x->w[i]) return 1;
  if (b & 63) return (xm_get(x, li) & ((1ULL << (b & 63)) - 1)) != 0;
  return 0;
}

/* clear every bit at position >= b */
static void xm_clear_from(xmag *x, int b) {
  int li = b >> 6;
  if (xm_empty(x)) return;
  if (li <= x->hi) {
    if (li >= x->lo) x->w[li] &= (b & 63) ? ((1ULL << (b & 63)) - 1) : 0;
    if (li + 1 <= x->hi) x->hi = li;
  }
  if (x->hi > li) x->hi = li;
  xm_trim(x);
}

/* x := 2^s - x, for 0 < x < 2^s */
static void xm_neg_field(xmag *x, int s) {
  int top = (s - 1) >> 6;
  xm_touch(x, x->lo, top);
  int i = x->lo;
  while (i <= top && x->w[i] == 0) i++;
  if (i > top) return; /* x == 0: not reached */
  x->w[i] = (uint64_t)(-(int64_t)x->w[i]);
  for (i = i + 1; i <= top; i++) x->w[i] = ~x->w[i];
  if (s & 63) x->w[top] &= (1ULL << (s & 63)) - 1;
  xm_trim(x);
}

static int xm_cmp(const xmag *a, const xmag *b) {
  int hi = a->hi > b->hi ? a->hi : b->hi;
  int lo = a->lo < b->lo ? a->lo : b->lo;
  for (int i = hi; i >= lo; i--) {
    uint64_t u = xm_get(a, i), v = xm_get(b, i);
    if (u != v) return u > v ? 1 : -1;
  }
  return 0;
}

/* d = a - b, requires a >= b */
static void xm_sub(const xmag *a, const xmag *b, xmag *d) {
  xm_clear(d);
  if (xm_empty(a)) return;
  int lo = a->lo, hi = a->hi;
  if (!xm_empty(b) && b->lo < lo) lo = b->lo;
  xm_touch(d, lo, hi);
  uint64_t br = 0;
  for (int i = lo; i <= hi; i++) {
    uint64_t u = xm_get(a, i), v = xm_get(b, i);
    u128 t = (u128)u - v - br;
    d->w[i] = (uint64_t)t;
    br = (uint64_t)(t >> 64) ? 1 : 0;
  }
  xm_trim(d);
}

/* d = a * 2^s, s >= 0 */
static void xm_shl(const xmag *a, int s, xmag *d) {
  xm_clear(d);
  if (xm_empty(a)) return;
  int q = s >> 6, r = s & 63;
  int lo = a->lo + q, hi = a->hi + q + 1;
  if (hi >= XW) hi = XW - 1;
  xm_touch(d, lo, hi);
  for (int i = lo; i <= hi; i++) {
    uint64_t cur = xm_get(a, i - q);
    uint64_t prev = xm_get(a, i - q - 1);
    d->w[i] = r ? ((cur << r) | (prev >> (64 - r))) : cur;
  }
  xm_trim(d);
}

/* ------------------------------------------------------------------------------------ */
/* Exact accumulator: positive and negative parts kept apart, so adding never borrows.   */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  xmag p, n;
  int bad; /* a NaN or infinity was added */
} xacc;

static inline void xa_clear(xacc *a) {
  xm_clear(&a->p);
  xm_clear(&a->n);
  a->bad = 0;
}

/* |d| = m * 2^e with m an integer below 2^53; returns the sign (0 for zero).
 * Read straight from the IEEE-754 fields: normal numbers carry the hidden bit,
 * subnormals (biased exponent 0) do not. */
static inline int dsplit(double d, uint64_t *m, int *e) {
  uint64_t u;
  memcpy(&u, &d, sizeof u);
  uint64_t frac = u & 0x000FFFFFFFFFFFFFULL;
  int bexp = (int)((u >> 52) & 0x7FF);
  if (bexp == 0) {
    if (frac == 0) return 0;
    *m = frac;
    *e = -1074;
  } else {
    *m = frac | 0x0010000000000000ULL;
    *e = bexp - 1075;
  }
  return (u >> 63) ? -1 : 1;
}

static inline void xa_add(xacc *a, double d) {
  if (!isfinite(d)) { a->bad = 1; return; }
  uint64_t m; int e;
  int s = dsplit(d, &m, &e);
  if (!s) return;
  xm_add_at(s > 0 ? &a->p : &a->n, (u128)m, e - XBASE);
}

/* a += x*y exactly */
static inline void xa_addmul(xacc *a, double x, double y) {
  if (!isfinite(x) || !isfinite(y)) { a->bad = 1; return; }
  uint64_t mx, my; int ex, ey;
  int sx = dsplit(x, &mx, &ex), sy = dsplit(y, &my, &ey);
  if (!sx || !sy) return;
  xm_add_at(sx * sy > 0 ? &a->p : &a->n, (u128)mx * my, ex + ey - XBASE);
}

/* d = |P - N|; returns sign(P - N) */
static int xa_resolve(const xacc *a, xmag *d) {
  int c = xm_cmp(&a->p, &a->n);
  if (c == 0) { xm_clear(d); return 0; }
  if (c > 0) xm_sub(&a->p, &a->n, d);
  else xm_sub(&a->n, &a->p, d);
  return c;
}

/* Greedy round-to-nearest of sign*|d| into C components. d is consumed. */
static void xm_round(xmag *d, int sign, int C, double *out) {
  for (int k = 0; k < C; k++) {
    int b = xm_msb(d);
    if (b < 0 || sign == 0 || b + XBASE < -1022) {
      for (; k < C; k++) out[k] = 0.0;
      return;
    }
    if (b + XBASE > 1023) {
      out[k] = sign > 0 ? INFINITY : -INFINITY;
      for (k = k + 1; k < C; k++) out[k] = 0.0;
      return;
    }
    int low = b - 52;
    uint64_t m = xm_bits(d, low, 53);
    int rb = xm_bit(d, low - 1);
    int st = xm_any_below(d, low - 1);
    int up = rb && (st || (m & 1u));
    double v = ldexp((double)(m + (uint64_t)up), low + XBASE);
    out[k] = sign > 0 ? v : -v;
    xm_clear_from(d, low);
    if (up) {
      xm_neg_field(d, low);
      sign = -sign;
    }
  }
}

static void xa_round(const xacc *a, int C, double *out) {
  if (a->bad) {
    for (int k = 0; k < C; k++) out[k] = NAN;
    return;
  }
  xmag d;
  int s = xa_resolve(a, &d);
  xm_round(&d, s, C, out);
}

/* exact sign of an accumulated sum */
static int xa_sign(const xacc *a) {
  xmag d;
  return xa_resolve(a, &d);
}

/* ------------------------------------------------------------------------------------ */
/* Real multi-component operations: each is exact-then-greedy-RN.                         */
/* ------------------------------------------------------------------------------------ */
static void mp_add(int C, const double *a, const double *b, double *o) {
  xacc x; xa_clear(&x);
  for (int k = 0; k < C; k++) { xa_add(&x, a[k]); xa_add(&x, b[k]); }
  xa_round(&x, C, o);
}

static void mp_sub(int C, const double *a, const double *b, double *o) {
  xacc x; xa_clear(&x);
  for (int k = 0; k < C; k++) { xa_add(&x, a[k]); xa_add(&x, -b[k]); }
  xa_round(&x, C, o);
}

static void mp_mul(int C, const double *a, const double *b, double *o) {
  xacc x; xa_clear(&x);
  for (int i = 0; i < C; i++)
    for (int j = 0; j < C; j++) xa_addmul(&x, a[i], b[j]);
  xa_round(&x, C, o);
}

/* RN(|R| / |B|) as a positive double; both nonzero */
static double rn_quot(const xmag *R, const xmag *B) {
  int br = xm_msb(R), bd = xm_msb(B);
  int shi = br - bd; /* quotient lies in [2^(shi-1), 2^(shi+1)) */
  int T = (shi - 57 < 0) ? 57 - shi : 0;
  xmag rem, tmp, bs;
  xm_shl(R, T, &rem);
  uint64_t Q = 0;
  for (int s = shi + T; s >= shi + T - 57; s--) {
    Q <<= 1;
    xm_shl(B, s, &bs);
    if (xm_cmp(&rem, &bs) >= 0) {
      xm_sub(&rem, &bs, &tmp);
      rem = tmp;
      Q |= 1;
    }
  }
  int sticky = xm_msb(&rem) >= 0;
  int top = 63 - __builtin_clzll(Q); /* 56 or 57 */
  int drop = top - 52;
  uint64_t m = Q >> drop;
  int rb = (int)((Q >> (drop - 1)) & 1u);
  sticky |= (Q & ((1ULL << (drop - 1)) - 1)) != 0;
  if (rb && (sticky || (m & 1u))) m++;
  return ldexp((double)m, drop + shi - 57);
}

/* o = a / b, greedily: q_k = RN((a - sum_{t<k} q_t b) / b) */
static void mp_div(int C, const double *a, const double *b, double *q) {
  xacc bb; xa_clear(&bb);
  for (int j = 0; j < C; j++) xa_add(&bb, b[j]);
  xmag B;
  int sb = xa_resolve(&bb, &B);
  if (sb == 0 || bb.bad) {
    for (int k = 0; k < C; k++) q[k] = NAN;
    return;
  }
  for (int k = 0; k < C; k++) {
    xacc r; xa_clear(&r);
    for (int j = 0; j < C; j++) xa_add(&r, a[j]);
    for (int t = 0; t < k; t++)
      for (int j = 0; j < C; j++) xa_addmul(&r, -q[t], b[j]);
    if (r.bad) { for (; k < C; k++) q[k] = NAN; return; }
    xmag R;
    int sr = xa_resolve(&r, &R);
    if (sr == 0) { for (; k < C; k++) q[k] = 0.0; return; }
    double v = rn_quot(&R, &B);
    if (v < 0x1p-1022) { for (; k < C; k++) q[k] = 0.0; return; }
    q[k] = (sr * sb > 0) ? v : -v;
  }
}

/* ------------------------------------------------------------------------------------ */
/* Complex values (real and imaginary parts kept apart, as in Sec. 2.2).                   */
/* ------------------------------------------------------------------------------------ */
typedef struct { double re[4], im[4]; } zmp;

static inline int z_iszero(int C, const zmp *a) {
  for (int k = 0; k < C; k++)
    if (a->re[k] != 0.0 || a->im[k] != 0.0) return 0;
  return 1;
}

/* 4M product, Eq. (4m): Re = Re(a)Re(b) - Im(a)Im(b), Im = Im(a)Re(b) + Re(a)Im(b).
 * Each real product is rounded, then the difference / sum is rounded. */
static void z_mul4m(int C, const zmp *a, const zmp *b, zmp *o) {
  double t1[4], t2[4], r[4], i_[4];
  mp_mul(C, a->re, b->re, t1);
  mp_mul(C, a->im, b->im, t2);
  mp_sub(C, t1, t2, r);
  mp_mul(C, a->im, b->re, t1);
  mp_mul(C, a->re, b->im, t2);
  mp_add(C, t1, t2, i_);
  memcpy(o->re, r, sizeof r);
  memcpy(o->im, i_, sizeof i_);
}

/* reciprocal 1/b = conj(b) / |b|^2 with |b|^2 = Re(b)^2 + Im(b)^2 rounded once */
static void z_recip(int C, const zmp *b, zmp *o) {
  xacc x; xa_clear(&x);
  for (int i = 0; i < C; i++)
    for (int j = 0; j < C; j++) {
      xa_addmul(&x, b->re[i], b->re[j]);
      xa_addmul(&x, b->im[i], b->im[j]);
    }
  double d[4], nim[4];
  xa_round(&x, C, d);
  for (int k = 0; k < C; k++) nim[k] = -b->im[k];
  zmp t;
  mp_div(C, b->re, d, t.re);
  mp_div(C, nim, d, t.im);
  *o = t;
}

/* a - p, per part */
static void z_sub(int C, const zmp *a, const zmp *p, zmp *o) {
  zmp t;
  mp_sub(C, a->re, p->re, t.re);
  mp_sub(C, a->im, p->im, t.im);
  *o = t;
}

static inline void z_conj(int C, zmp *a) {
  for (int k = 0; k < C; k++) a->im[k] = -a->im[k];
}

/* exact sign of the real sum of C components */
static int part_sign(int C, const double *v) {
  xacc x; xa_clear(&x);
  for (int k = 0; k < C; k++) xa_add(&x, v[k]);
  return xa_sign(&x);
}

/* sign(cabs1(x) - cabs1(y)) exactly, cabs1(z) = |Re z| + |Im z| (full precision) */
static int cabs1_cmp(int C, const zmp *x, const zmp *y) {
  int sxr = part_sign(C, x->re), sxi = part_sign(C, x->im);
  int syr = part_sign(C, y->re), syi = part_sign(C, y->im);
  xacc a; xa_clear(&a);
  for (int k = 0; k < C; k++) {
    xa_add(&a, sxr * x->re[k]);
    xa_add(&a, sxi * x->im[k]);
    xa_add(&a, -syr * y->re[k]);
    xa_add(&a, -syi * y->im[k]);
  }
  return xa_sign(&a);
}

/* ------------------------------------------------------------------------------------ */
/* Plane access helpers                                                                   */
/* ------------------------------------------------------------------------------------ */
static inline void ld_z(int C, const double *P, int64_t ld, int64_t ps, int64_t i, int64_t j,
                        zmp *z) {
  for (int c = 0; c < C; c++) {
    z->re[c] = P[(int64_t)c * ps + j * ld + i];
    z->im[c] = P[(int64_t)(C + c) * ps + j * ld + i];
  }
  for (int c = C; c < 4; c++) z->re[c] = z->im[c] = 0.0;
}

static inline void st_z(int C, double *P, int64_t ld, int64_t ps, int64_t i, int64_t j,
                        const zmp *z) {
  for (int c = 0; c < C; c++) {
    P[(int64_t)c * ps + j * ld + i] = z->re[c];
    P[(int64_t)(C + c) * ps + j * ld + i] = z->im[c];
  }
}

static int set_threads(int nthr) {
#ifdef _OPENMP
  if (nthr > 0) omp_set_num_threads(nthr);
  return omp_get_max_threads();
#else
  (void)nthr;
  return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* Exported entry points                                                                  */
/* ------------------------------------------------------------------------------------ */
int orc_version(void) { return 1; }

int orc_threads(int nthr) { return set_threads(nthr); }

/* scalar ops for the arithmetic pins; a, b, o are C-component arrays */
void orc_mp_add(int C, const double *a, const double *b, double *o) { mp_add(C, a, b, o); }
void orc_mp_sub(int C, const double *a, const double *b, double *o) { mp_sub(C, a, b, o); }
void orc_mp_mul(int C, const double *a, const double *b, double *o) { mp_mul(C, a, b, o); }
void orc_mp_div(int C, const double *a, const double *b, double *o) { mp_div(C, a, b, o); }

/* greedy RN of the exact sum of n doubles into C components */
void orc_mp_round(int C, int n, const double *v, double *o) {
  xacc x; xa_clear(&x);
  for (int k = 0; k < n; k++) xa_add(&x, v[k]);
  xa_round(&x, C, o);
}

/* complex scalar ops: inputs/outputs as [re_0..re_{C-1}, im_0..im_{C-1}] */
static void unpack(int C, const double *v, zmp *z) {
  memset(z, 0, sizeof *z);
  for (int c = 0; c < C; c++) { z->re[c] = v[c]; z->im[c] = v[C + c]; }
}
static void pack(int C, const zmp *z, double *v) {
  for (int c = 0; c < C; c++) { v[c] = z->re[c]; v[C + c] = z->im[c]; }
}
void orc_z_mul4m(int C, const double *a, const double *b, double *o) {
  zmp x, y, r; unpack(C, a, &x); unpack(C, b, &y); z_mul4m(C, &x, &y, &r); pack(C, &r, o);
}
void orc_z_recip(int C, const double *a, double *o) {
  zmp x, r; unpack(C, a, &x); z_recip(C, &x, &r); pack(C, &r, o);
}
int orc_z_cabs1_cmp(int C, const double *a, const double *b) {
  zmp x, y; unpack(C, a, &x); unpack(C, b, &y); return cabs1_cmp(C, &x, &y);
}

/* Canonicalise in place: every element becomes the greedy RN of its exact value. */
int orc_zcanon(int C, int64_t m, int64_t n, double *A, int64_t ld, int64_t ps) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; j++)
    for (int64_t i = 0; i < m; i++)
      for (int ri = 0; ri < 2; ri++) {
        double v[4], o[4];
        for (int c = 0; c < C; c++) v[c] = A[(int64_t)(ri * C + c) * ps + j * ld + i];
        orc_mp_round(C, C, v, o);
        for (int c = 0; c < C; c++) A[(int64_t)(ri * C + c) * ps + j * ld + i] = o[c];
      }
  return 0;
}

/* Convert between precisions: B (Cout comps) = greedy RN of exact A (Cin comps). */
int orc_zround(int Cin, int Cout, int64_t m, int64_t n, const double *A, int64_t lda,
               int64_t psa, double *B, int64_t ldb, int64_t psb) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; j++)
    for (int64_t i = 0; i < m; i++)
      for (int ri = 0; ri < 2; ri++) {
        double v[4], o[4];
        for (int c = 0; c < Cin; c++) v[c] = A[(int64_t)(ri * Cin + c) * psa + j * lda + i];
        orc_mp_round(Cout, Cin, v, o);
        for (int c = 0; c < Cout; c++) B[(int64_t)(ri * Cout + c) * psb + j * ldb + i] = o[c];
      }
  return 0;
}

/* Elementwise exact difference rounded to one double: D = RN(X - Y). */
int orc_zdiff(int CX, int CY, int64_t m, int64_t n, const double *X, int64_t ldx, int64_t psx,
              const double *Y, int64_t ldy, int64_t psy, double *Dre, double *Dim) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; j++)
    for (int64_t i = 0; i < m; i++)
      for (int ri = 0; ri < 2; ri++) {
        xacc x; xa_clear(&x);
        for (int c = 0; c < CX; c++) xa_add(&x, X[(int64_t)(ri * CX + c) * psx + j * ldx + i]);
        for (int c = 0; c < CY; c++) xa_add(&x, -Y[(int64_t)(ri * CY + c) * psy + j * ldy + i]);
        double o[1];
        xa_round(&x, 1, o);
        (ri ? Dim : Dre)[j * m + i] = o[0];
      }
  return 0;
}

/*
 * Unblocked right-looking LU with partial pivoting, the paper's "Normal LU" (Sec. 3),
 * with LAPACK getf2 conventions and 4M complex arithmetic (Eq. 4m).  For k = 0, 1, ...:
 *   p = first row i >= k maximising cabs1(A[i,k]) = |Re| + |Im| (exact comparison);
 *   ipiv[k] = p + 1;
 *   if A[p,k] != 0: swap rows k and p across all n columns; r = 1/A[k,k];
 *                   A[i,k] = A[i,k] * r for i > k;
 *   else if info == 0: info = k + 1;
 *   A[i,j] = A[i,j] - (A[i,k] * A[k,j]) for i > k, j > k (product rounded, then the sub).
 * kmax < min(m,n) stops after kmax columns (used to time a bounded sample).
 */
int orc_zgetf2(int C, int64_t m, int64_t n, double *A, int64_t ld, int64_t ps, int32_t *ipiv,
               int32_t *info, int64_t kmax, int nthr) {
  if (C < 2 || C > 4 || m < 0 || n < 0 || ld < (m > 1 ? m : 1)) return -1;
  set_threads(nthr);
  int64_t mn = m < n ? m : n;
  if (kmax < 0 || kmax > mn) kmax = mn;
  zmp *M = (zmp *)malloc(sizeof(zmp) * (size_t)(m > 0 ? m : 1) * (size_t)(n > 0 ? n : 1));
  if (!M) return -2;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; j++)
    for (int64_t i = 0; i < m; i++) ld_z(C, A, ld, ps, i, j, &M[j * m + i]);
  *info = 0;
  for (int64_t k = 0; k < kmax; k++) {
    int64_t p = k;
    for (int64_t i = k + 1; i < m; i++)
      if (cabs1_cmp(C, &M[k * m + i], &M[k * m + p]) > 0) p = i;
    ipiv[k] = (int32_t)(p + 1);
    if (!z_iszero(C, &M[k * m + p])) {
      if (p != k)
        for (int64_t j = 0; j < n; j++) {
          zmp t = M[j * m + k];
          M[j * m + k] = M[j * m + p];
          M[j * m + p] = t;
        }
      zmp r;
      z_recip(C, &M[k * m + k], &r);
#pragma omp parallel for schedule(static)
      for (int64_t i = k + 1; i < m; i++) z_mul4m(C, &M[k * m + i], &r, &M[k * m + i]);
    } else if (*info == 0) {
      *info = (int32_t)(k + 1);
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = k + 1; i < m; i++) {
      const zmp *l = &M[k * m + i];
      for (int64_t j = k + 1; j < n; j++) {
        zmp prod;
        z_mul4m(C, l, &M[j * m + k], &prod);
        z_sub(C, &M[j * m + i], &prod, &M[j * m + i]);
      }
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; j++)
    for (int64_t i = 0; i < m; i++) st_z(C, A, ld, ps, i, j, &M[j * m + i]);
  free(M);
  return 0;
}

/*
 * Forward and backward substitution with the factors of orc_zgetf2 (Sec. 4 solves with
 * them).  trans 'N': apply the swaps in order, y_i = b_i - sum_{k<i} L_ik y_k (k ascending,
 * unit diagonal), then x_i = (y_i - sum_{k>i} U_ik x_k) * (1/U_ii) (k descending).
 * trans 'C' solves A^H x = b: U^H z = b (forward), L^H w = z (backward), then the swaps
 * in reverse order.  Each accumulation step is one rounded 4M product and one rounded sub.
 */
int orc_zgetrs(int C, char trans, int64_t n, int64_t nrhs, const double *LU, int64_t ld,
               int64_t ps, const int32_t *ipiv, double *B, int64_t ldb, int64_t psb, int nthr) {
  if (C < 2 || C > 4 || (trans != 'N' && trans != 'C')) return -1;
  set_threads(nthr);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nrhs; r++) {
    zmp *x = (zmp *)malloc(sizeof(zmp) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) ld_z(C, B, ldb, psb, i, r, &x[i]);
    zmp l, u, prod, rc;
    if (trans == 'N') {
      for (int64_t k = 0; k < n; k++) {
        int64_t p = ipiv[k] - 1;
        if (p != k) { zmp t = x[k]; x[k] = x[p]; x[p] = t; }
      }
      for (int64_t i = 0; i < n; i++)
        for (int64_t k = 0; k < i; k++) {
          ld_z(C, LU, ld, ps, i, k, &l);
          z_mul4m(C, &l, &x[k], &prod);
          z_sub(C, &x[i], &prod, &x[i]);
        }
      for (int64_t i = n - 1; i >= 0; i--) {
        for (int64_t k = n - 1; k > i; k--) {
          ld_z(C, LU, ld, ps, i, k, &u);
          z_mul4m(C, &u, &x[k], &prod);
          z_sub(C, &x[i], &prod, &x[i]);
        }
        ld_z(C, LU, ld, ps, i, i, &u);
        z_recip(C, &u, &rc);
        z_mul4m(C, &x[i], &rc, &x[i]);
      }
    } else {
      for (int64_t i = 0; i < n; i++) {
        for (int64_t k = 0; k < i; k++) {
          ld_z(C, LU, ld, ps, k, i, &u);
          z_conj(C, &u);
          z_mul4m(C, &u, &x[k], &prod);
          z_sub(C, &x[i], &prod, &x[i]);
        }
        ld_z(C, LU, ld, ps, i, i, &u);
        z_conj(C, &u);
        z_recip(C, &u, &rc);
        z_mul4m(C, &x[i], &rc, &x[i]);
      }
      for (int64_t i = n - 1; i >= 0; i--)
        for (int64_t k = n - 1; k > i; k--) {
          ld_z(C, LU, ld, ps, k, i, &l);
          z_conj(C, &l);
          z_mul4m(C, &l, &x[k], &prod);
          z_sub(C, &x[i], &prod, &x[i]);
        }
      for (int64_t k = n - 1; k >= 0; k--) {
        int64_t p = ipiv[k] - 1;
        if (p != k) { zmp t = x[k]; x[k] = x[p]; x[p] = t; }
      }
    }
    for (int64_t i = 0; i < n; i++) st_z(C, B, ldb, psb, i, r, &x[i]);
    free(x);
  }
  return 0;
}

/* element (i,t) of op(A): 'N' A[i,t], 'T' A[t,i], 'C' conj(A[t,i]) */
static inline void ld_op(int C, char op, const double *A, int64_t ld, int64_t ps, int64_t i,
                         int64_t t, zmp *z) {
  if (op == 'N') ld_z(C, A, ld, ps, i, t, z);
  else {
    ld_z(C, A, ld, ps, t, i, z);
    if (op == 'C') z_conj(C, z);
  }
}

/*
 * Complex matrix product  Cm := beta*Cm + alpha*op(A)*op(B),  alpha = +-1, beta in {0,1}.
 * method 4 (Eq. 4m): each part of the exact product is rounded once,
 *   Re = RN(ReA.ReB - ImA.ImB),  Im = RN(ImA.ReB + ReA.ImB).
 * method 3 (Eq. 3m_cemm): the three real products T1 = ReA.ReB, T2 = ImA.ImB and
 *   T3 = (ReA+ImA).(ReB+ImB) are each exact dot products rounded once (the two sums are
 *   rounded elementwise first); then Re = RN(T1 - T2), Im = RN(RN(T3 - T1) - T2).
 * The result is then added to (beta=1) or stored in (beta=0) Cm, rounded once.
 */
int orc_zgemm(int C, int method, char opA, char opB, int64_t m, int64_t n, int64_t k,
              int alpha_sign, const double *A, int64_t lda, int64_t psa, const double *B,
              int64_t ldb, int64_t psb, int beta, double *Cm, int64_t ldc, int64_t psc,
              int nthr) {
  if (C < 2 || C > 4 || (method != 3 && method != 4)) return -1;
  set_threads(nthr);
  /* op(A) is m x k, op(B) is k x n; unpack both */
  zmp *Aop = (zmp *)malloc(sizeof(zmp) * (size_t)(m * k > 0 ? m * k : 1));
  zmp *Bop = (zmp *)malloc(sizeof(zmp) * (size_t)(k * n > 0 ? k * n : 1));
  for (int64_t i = 0; i < m; i++)
    for (int64_t t = 0; t < k; t++) ld_op(C, opA, A, lda, psa, i, t, &Aop[i * k + t]);
  for (int64_t t = 0; t < k; t++)
    for (int64_t j = 0; j < n; j++) ld_op(C, opB, B, ldb, psb, t, j, &Bop[j * k + t]);
  double *SA = NULL, *SB = NULL;
  if (method == 3) {
    SA = (double *)malloc(sizeof(double) * 4 * (size_t)(m * k > 0 ? m * k : 1));
    SB = (double *)malloc(sizeof(double) * 4 * (size_t)(k * n > 0 ? k * n : 1));
    for (int64_t e = 0; e < m * k; e++) mp_add(C, Aop[e].re, Aop[e].im, &SA[4 * e]);
    for (int64_t e = 0; e < k * n; e++) mp_add(C, Bop[e].re, Bop[e].im, &SB[4 * e]);
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < m; i++) {
    for (int64_t j = 0; j < n; j++) {
      zmp res, cur;
      double t1[4], t2[4], t3[4], tmp[4];
      xacc x;
      const zmp *a = &Aop[i * k], *b = &Bop[j * k];
      if (method == 4) {
        xa_clear(&x);
        for (int64_t t = 0; t < k; t++)
          for (int p = 0; p < C; p++)
            for (int q = 0; q < C; q++) {
              xa_addmul(&x, a[t].re[p], b[t].re[q]);
              xa_addmul(&x, -a[t].im[p], b[t].im[q]);
            }
        xa_round(&x, C, res.re);
        xa_clear(&x);
        for (int64_t t = 0; t < k; t++)
          for (int p = 0; p < C; p++)
            for (int q = 0; q < C; q++) {
              xa_addmul(&x, a[t].im[p], b[t].re[q]);
              xa_addmul(&x, a[t].re[p], b[t].im[q]);
            }
        xa_round(&x, C, res.im);
      } else {
        const double *sa = &SA[4 * i * k], *sb = &SB[4 * j * k];
        xa_clear(&x);
        for (int64_t t = 0; t < k; t++)
          for (int p = 0; p < C; p++)
            for (int q = 0; q < C; q++) xa_addmul(&x, a[t].re[p], b[t].re[q]);
        xa_round(&x, C, t1);
        xa_clear(&x);
        for (int64_t t = 0; t < k; t++)
          for (int p = 0; p < C; p++)
            for (int q = 0; q < C; q++) xa_addmul(&x, a[t].im[p], b[t].im[q]);
        xa_round(&x, C, t2);
        xa_clear(&x);
        for (int64_t t = 0; t < k; t++)
          for (int p = 0; p < C; p++)
            for (int q = 0; q < C; q++) xa_addmul(&x, sa[4 * t + p], sb[4 * t + q]);
        xa_round(&x, C, t3);
        mp_sub(C, t1, t2, res.re);
        mp_sub(C, t3, t1, tmp);
        mp_sub(C, tmp, t2, res.im);
      }
      if (alpha_sign < 0)
        for (int c = 0; c < C; c++) { res.re[c] = -res.re[c]; res.im[c] = -res.im[c]; }
      if (beta) {
        ld_z(C, Cm, ldc, psc, i, j, &cur);
        mp_add(C, cur.re, res.re, res.re);
        mp_add(C, cur.im, res.im, res.im);
      }
      st_z(C, Cm, ldc, psc, i, j, &res);
    }
  }
  free(Aop); free(Bop); free(SA); free(SB);
  return 0;
}

/* Exact product rounded once per part: Bout = RN(A * X)  (A m x n, X n x nrhs). */
int orc_zmatmul_exact(int C, int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                      int64_t psa, const double *X, int64_t ldx, int64_t psx, double *Bo,
                      int64_t ldb, int64_t psb, int nthr) {
  set_threads(nthr);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < m; i++)
    for (int64_t r = 0; r < nrhs; r++) {
      xacc xr, xi;
      xa_clear(&xr); xa_clear(&xi);
      zmp a, x;
      for (int64_t j = 0; j < n; j++) {
        ld_z(C, A, lda, psa, i, j, &a);
        ld_z(C, X, ldx, psx, j, r, &x);
        for (int p = 0; p < C; p++)
          for (int q = 0; q < C; q++) {
            xa_addmul(&xr, a.re[p], x.re[q]);
            xa_addmul(&xr, -a.im[p], x.im[q]);
            xa_addmul(&xi, a.re[p], x.im[q]);
            xa_addmul(&xi, a.im[p], x.re[q]);
          }
      }
      zmp o;
      xa_round(&xr, C, o.re);
      xa_round(&xi, C, o.im);
      st_z(C, Bo, ldb, psb, i, r, &o);
    }
  return 0;
}

/* Exact residual r = b - A x rounded once to double per part (CA, CX, CB components). */
int orc_zresid(int CA, int CX, int CB, int64_t n, int64_t nrhs, const double *A, int64_t lda,
               int64_t psa, const double *X, int64_t ldx, int64_t psx, const double *Bv,
               int64_t ldb, int64_t psb, double *Rre, double *Rim, int nthr) {
  set_threads(nthr);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; i++)
    for (int64_t r = 0; r < nrhs; r++) {
      xacc xr, xi;
      xa_clear(&xr); xa_clear(&xi);
      for (int c = 0; c < CB; c++) {
        xa_add(&xr, Bv[(int64_t)c * psb + r * ldb + i]);
        xa_add(&xi, Bv[(int64_t)(CB + c) * psb + r * ldb + i]);
      }
      for (int64_t j = 0; j < n; j++)
        for (int p = 0; p < CA; p++) {
          double ar = A[(int64_t)p * psa + j * lda + i];
          double ai = A[(int64_t)(CA + p) * psa + j * lda + i];
          for (int q = 0; q < CX; q++) {
            double xr_ = X[(int64_t)q * psx + r * ldx + j];
            double xi_ = X[(int64_t)(CX + q) * psx + r * ldx + j];
            xa_addmul(&xr, -ar, xr_);
            xa_addmul(&xr, ai, xi_);
            xa_addmul(&xi, -ar, xi_);
            xa_addmul(&xi, -ai, xr_);
          }
        }
      double o[1];
      xa_round(&xr, 1, o);
      Rre[r * n + i] = o[0];
      xa_round(&xi, 1, o);
      Rim[r * n + i] = o[0];
    }
  return 0;
}

/*
 * Ill-conditioned test matrix A = U diag(sigma) V^H, U and V each a product of nrefl
 * complex Householder reflectors H = I - tau v v^H, tau = 2/(v^H v), v given as exact
 * doubles (the caller draws them).  sigma: n values of C components (real).
 * VL, VR: nrefl*n complex doubles as [t][re/im][i] (re at t*2n + i, im at t*2n + n + i).
 * Order: M = diag(sigma); M = M H'_t for t = nrefl-1 .. 0; then M = H_t M for
 * t = nrefl-1 .. 0.  Each updated element is one exact expression rounded once.
 */
int orc_gen_illcond(int C, int64_t n, const double *sigma, int nrefl, const double *VL,
                    const double *VR, double *A, int64_t ld, int64_t ps, int nthr) {
  set_threads(nthr);
  zmp *M = (zmp *)calloc((size_t)(n * n > 0 ? n * n : 1), sizeof(zmp));
  zmp *w = (zmp *)calloc((size_t)(n > 0 ? n : 1), sizeof(zmp));
  if (!M || !w) { free(M); free(w); return -2; }
  for (int64_t i = 0; i < n; i++)
    for (int c = 0; c < C; c++) M[i * n + i].re[c] = sigma[i * C + c];
  for (int side = 0; side < 2; side++) {
    const double *V = side == 0 ? VR : VL;
    for (int t = nrefl - 1; t >= 0; t--) {
      const double *vr = V + (int64_t)t * 2 * n, *vi = vr + n;
      /* tau = 2 / (v^H v) */
      double vv[4], two[4] = {2.0, 0, 0, 0}, tau[4];
      {
        xacc x; xa_clear(&x);
        for (int64_t i = 0; i < n; i++) { xa_addmul(&x, vr[i], vr[i]); xa_addmul(&x, vi[i], vi[i]); }
        xa_round(&x, C, vv);
      }
      mp_div(C, two, vv, tau);
      if (side == 0) {
        /* right: M = M - tau (M v) v^H ;  w_i = sum_j M_ij v_j  (M stored row-major here) */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) {
          xacc xr, xi; xa_clear(&xr); xa_clear(&xi);
          for (int64_t j = 0; j < n; j++) {
            const zmp *mm = &M[i * n + j];
            for (int c = 0; c < C; c++) {
              xa_addmul(&xr, mm->re[c], vr[j]); xa_addmul(&xr, -mm->im[c], vi[j]);
              xa_addmul(&xi, mm->re[c], vi[j]); xa_addmul(&xi, mm->im[c], vr[j]);
            }
          }
          double a[4], b[4];
          xa_round(&xr, C, a); xa_round(&xi, C, b);
          mp_mul(C, a, tau, w[i].re); mp_mul(C, b, tau, w[i].im);
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++)
          for (int64_t j = 0; j < n; j++) {
            /* M_ij -= w_i * conj(v_j) */
            zmp *mm = &M[i * n + j];
            xacc xr, xi; xa_clear(&xr); xa_clear(&xi);
            for (int c = 0; c < C; c++) {
              xa_add(&xr, mm->re[c]); xa_add(&xi, mm->im[c]);
              xa_addmul(&xr, -w[i].re[c], vr[j]); xa_addmul(&xr, -w[i].im[c], vi[j]);
              xa_addmul(&xi, -w[i].im[c], vr[j]); xa_addmul(&xi, w[i].re[c], vi[j]);
            }
            xa_round(&xr, C, mm->re); xa_round(&xi, C, mm->im);
          }
      } else {
        /* left: M = M - tau v (v^H M) ;  w_j = sum_i conj(v_i) M_ij */
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; j++) {
          xacc xr, xi; xa_clear(&xr); xa_clear(&xi);
          for (int64_t i = 0; i < n; i++) {
            const zmp *mm = &M[i * n + j];
            for (int c = 0; c < C; c++) {
              xa_addmul(&xr, mm->re[c], vr[i]); xa_addmul(&xr, mm->im[c], vi[i]);
              xa_addmul(&xi, mm->im[c], vr[i]); xa_addmul(&xi, -mm->re[c], vi[i]);
            }
          }
          double a[4], b[4];
          xa_round(&xr, C, a); xa_round(&xi, C, b);
          mp_mul(C, a, tau, w[j].re); mp_mul(C, b, tau, w[j].im);
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++)
          for (int64_t j = 0; j < n; j++) {
            /* M_ij -= v_i * w_j */
            zmp *mm = &M[i * n + j];
            xacc xr, xi; xa_clear(&xr); xa_clear(&xi);
            for (int c = 0; c < C; c++) {
              xa_add(&xr, mm->re[c]); xa_add(&xi, mm->im[c]);
              xa_addmul(&xr, -vr[i], w[j].re[c]); xa_addmul(&xr, vi[i], w[j].im[c]);
              xa_addmul(&xi, -vr[i], w[j].im[c]); xa_addmul(&xi, -vi[i], w[j].re[c]);
            }
            xa_round(&xr, C, mm->re); xa_round(&xi, C, mm->im);
          }
      }
    }
  }
  for (int64_t i = 0; i < n; i++)
    for (int64_t j = 0; j < n; j++) st_z(C, A, ld, ps, i, j, &M[i * n + j]);
  free(M); free(w);
  return 0;
}
