// mp.hpp -- device-side multi-component floating-point arithmetic for gfx950.
//
// A real value is an unevaluated sum of C binary64 components (C = 2 double-double,
// 3 triple-double, 4 quadruple-double; Kouya Sec. 1).  All routines are built on the
// error-free transformations TwoSum (Knuth), FastTwoSum (Dekker) and TwoProd through a
// fused multiply-add; the library is compiled with floating-point contraction off so
// that the compiler neither fuses nor reassociates them.
//
// "Level accumulator": an array l[C] holding a value as sum(l) where l[o] collects terms
// of magnitude about 2^(-53 o) relative to the leading level.  A term pushed into level
// o < C-1 goes through TwoSum and its rounding error is pushed into level o+1; the last
// level is a plain sum.  Accumulating sums of products this way keeps every level
// exact except the last, so a K-term dot product has an error of order K u |a||b| with
// u = 2^(-53 C) as long as the levels are re-levelled (tidy) every few pushes in long
// sums; the value is renormalised to non-overlapping components only when it is stored (this is the accumulation scheme of Ogita, Rump and Oishi's Dot2 applied per
// level).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace mp {

__host__ __device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__host__ __device__ __forceinline__ void two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}

// push term t into level o of a C-level accumulator (cascade of TwoSum errors)
template <int C>
__host__ __device__ __forceinline__ void push(double (&l)[C], int o, double t) {
#pragma unroll
  for (int k = 0; k < C - 1; ++k) {
    if (k >= o) {
      double s, e;
      two_sum(l[k], t, s, e);
      l[k] = s;
      t = e;
    }
  }
  l[C - 1] += t;
}

// push a C-component value (component k at level k)
template <int C>
__host__ __device__ __forceinline__ void push_mp(double (&l)[C], const double (&v)[C]) {
#pragma unroll
  for (int k = 0; k < C; ++k) push<C>(l, k, v[k]);
}

template <int C>
__host__ __device__ __forceinline__ void push_mp_neg(double (&l)[C], const double (&v)[C]) {
#pragma unroll
  for (int k = 0; k < C; ++k) push<C>(l, k, -v[k]);
}

// l += a*b (a, b C-component values).  Products a_i b_j of order i+j < C-1 are split by
// TwoProd; the rounding error of an order-o product is a term of level o+1.  Order C-1
// products and level C-1 terms are gathered by a fused multiply-add chain.
template <int C>
__host__ __device__ __forceinline__ void mac(double (&l)[C], const double (&a)[C], const double (&b)[C]) {
  double last = 0.0;
  bool have = false;
#pragma unroll
  for (int o = 0; o < C - 1; ++o) {
#pragma unroll
    for (int i = 0; i <= o; ++i) {
      double p, e;
      two_prod(a[i], b[o - i], p, e);
      push<C>(l, o, p);
      if (o + 1 == C - 1) {
        if (have) last += e;
        else { last = e; have = true; }
      } else {
        push<C>(l, o + 1, e);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < C; ++i) {
    if (have) last = __builtin_fma(a[i], b[C - 1 - i], last);
    else { last = a[i] * b[C - 1 - i]; have = true; }
  }
  l[C - 1] += last;
}

// l += a * s for a C-component a and a binary64 s
template <int C>
__host__ __device__ __forceinline__ void mac_scalar(double (&l)[C], const double (&a)[C], double s) {
#pragma unroll
  for (int i = 0; i < C - 1; ++i) {
    double p, e;
    two_prod(a[i], s, p, e);
    push<C>(l, i, p);
    push<C>(l, i + 1, e);
  }
  l[C - 1] = __builtin_fma(a[C - 1], s, l[C - 1]);
}

// Re-level an accumulator in place, exactly: one bottom-up chain of TwoSum leaves the
// value unchanged and each level again about the rounding error of the level above.
// Long accumulations call it every few pushes.  Without it, when the leading level keeps
// growing (a sum of same-sign terms), every push hands the next level an error of half an
// ulp of the grown leading level; those errors pile up, and for C >= 3 the plain last
// level then rounds relative to the piled-up size, so an n-term sum loses accuracy faster
// than n u.
template <int C>
__host__ __device__ __forceinline__ void tidy(double (&l)[C]) {
#pragma unroll
  for (int k = C - 1; k > 0; --k) {
    double s, e;
    two_sum(l[k - 1], l[k], s, e);
    l[k - 1] = s;
    l[k] = e;
  }
}

// Renormalise a level accumulator into non-overlapping components.  Each pass is a
// full bottom-up chain of TwoSum (an error-free "VecSum": the exact sum is preserved and
// its rounded value lands on top); repeating the pass C-1 times re-merges what a
// cancellation between levels leaves behind, so the result is non-overlapping even when
// the levels cancel each other.  Leading zeros are squeezed out at the end.  For C = 2
// one TwoSum already gives |lo| <= ulp(hi)/2.
template <int C>
__host__ __device__ __forceinline__ void renorm(const double (&l)[C], double (&o)[C]) {
  double v[C];
#pragma unroll
  for (int k = 0; k < C; ++k) v[k] = l[k];
#pragma unroll
  for (int p = 0; p < (C == 2 ? 1 : C); ++p) {
#pragma unroll
    for (int k = C - 1; k > 0; --k) {
      double s, e;
      two_sum(v[k - 1], v[k], s, e);
      v[k - 1] = s;
      v[k] = e;
    }
  }
#pragma unroll
  for (int r = 0; r < C - 1; ++r) {
    // if v[r] == 0, shift the tail up by one
    bool z = (v[r] == 0.0);
#pragma unroll
    for (int k = r; k < C - 1; ++k) v[k] = z ? v[k + 1] : v[k];
    v[C - 1] = z ? 0.0 : v[C - 1];
  }
#pragma unroll
  for (int k = 0; k < C; ++k) o[k] = v[k];
}

template <int C>
__host__ __device__ __forceinline__ void set_zero(double (&v)[C]) {
#pragma unroll
  for (int k = 0; k < C; ++k) v[k] = 0.0;
}

template <int C>
__host__ __device__ __forceinline__ void copy(const double (&a)[C], double (&o)[C]) {
#pragma unroll
  for (int k = 0; k < C; ++k) o[k] = a[k];
}

template <int C>
__host__ __device__ __forceinline__ void neg(const double (&a)[C], double (&o)[C]) {
#pragma unroll
  for (int k = 0; k < C; ++k) o[k] = -a[k];
}

template <int C>
__host__ __device__ __forceinline__ bool is_zero(const double (&a)[C]) {
  bool z = true;
#pragma unroll
  for (int k = 0; k < C; ++k) z = z && (a[k] == 0.0);
  return z;
}

// a + b (error of order u (|a| + |b|))
template <int C>
__host__ __device__ __forceinline__ void add(const double (&a)[C], const double (&b)[C], double (&o)[C]) {
  double l[C];
  copy<C>(a, l);
  push_mp<C>(l, b);
  renorm<C>(l, o);
}

template <int C>
__host__ __device__ __forceinline__ void sub(const double (&a)[C], const double (&b)[C], double (&o)[C]) {
  double l[C];
  copy<C>(a, l);
  push_mp_neg<C>(l, b);
  renorm<C>(l, o);
}

template <int C>
__host__ __device__ __forceinline__ void mul(const double (&a)[C], const double (&b)[C], double (&o)[C]) {
  double l[C];
  set_zero<C>(l);
  mac<C>(l, a, b);
  renorm<C>(l, o);
}

// sign of a renormalised value: the sign of its first non-zero component
template <int C>
__host__ __device__ __forceinline__ int sign(const double (&a)[C]) {
  int s = 0;
#pragma unroll
  for (int k = C - 1; k >= 0; --k) s = (a[k] > 0.0) ? 1 : ((a[k] < 0.0) ? -1 : s);
  return s;
}

template <int C>
__host__ __device__ __forceinline__ void abs_(const double (&a)[C], double (&o)[C]) {
  bool n = sign<C>(a) < 0;
#pragma unroll
  for (int k = 0; k < C; ++k) o[k] = n ? -a[k] : a[k];
}

// sign(a - b)
template <int C>
__host__ __device__ __forceinline__ int cmp(const double (&a)[C], const double (&b)[C]) {
  double d[C];
  sub<C>(a, b, d);
  return sign<C>(d);
}

// 1/d by long division: q_t = r_0 / d_0 with the remainder r = 1 - (q_0 + ... ) d kept
// in a level accumulator; C + 1 quotient terms are summed and renormalised.
template <int C>
__host__ __device__ __forceinline__ void recip(const double (&d)[C], double (&o)[C]) {
  double r[C];
  set_zero<C>(r);
  r[0] = 1.0;
  double q[C];
  set_zero<C>(q);
  double rn[C];
#pragma unroll
  for (int t = 0; t <= C; ++t) {
    renorm<C>(r, rn);
    copy<C>(rn, r);  // keep the remainder non-overlapping so rn[0] leads it
    double qt = rn[0] / d[0];
    double nd[C];
    neg<C>(d, nd);
    mac_scalar<C>(r, nd, qt);
    push<C>(q, t < C ? t : C - 1, qt);
  }
  renorm<C>(q, o);
}

// ----------------------------------------------------------------------- complex ops
// complex value: re[C], im[C]

// o = a - l * u  (4M, Eq. 4m), one rounding per part
template <int C>
__host__ __device__ __forceinline__ void zfms(const double (&ar)[C], const double (&ai)[C],
                                     const double (&lr)[C], const double (&li)[C],
                                     const double (&ur)[C], const double (&ui)[C],
                                     double (&or_)[C], double (&oi)[C]) {
  double nlr[C], nli[C];
  neg<C>(lr, nlr);
  neg<C>(li, nli);
  double xr[C], xi[C];
  copy<C>(ar, xr);
  copy<C>(ai, xi);
  mac<C>(xr, nlr, ur);  // - lr ur
  mac<C>(xr, li, ui);   // + li ui
  mac<C>(xi, nlr, ui);  // - lr ui
  mac<C>(xi, nli, ur);  // - li ur
  renorm<C>(xr, or_);
  renorm<C>(xi, oi);
}

// o = a * b (4M), one rounding per part
template <int C>
__host__ __device__ __forceinline__ void zmul(const double (&ar)[C], const double (&ai)[C],
                                     const double (&br)[C], const double (&bi)[C],
                                     double (&or_)[C], double (&oi)[C]) {
  double nai[C];
  neg<C>(ai, nai);
  double xr[C], xi[C];
  set_zero<C>(xr);
  set_zero<C>(xi);
  mac<C>(xr, ar, br);
  mac<C>(xr, nai, bi);
  mac<C>(xi, ar, bi);
  mac<C>(xi, ai, br);
  renorm<C>(xr, or_);
  renorm<C>(xi, oi);
}

// 2^-e for the exponent e of the larger leading component of b (clamped so that the scale
// stays a normal number); 1 for zero, infinite or NaN leading components
__host__ __device__ __forceinline__ double recip_scale(double r0, double i0) {
  const double m = fabs(r0) > fabs(i0) ? fabs(r0) : fabs(i0);
  const long long bits = __builtin_bit_cast(long long, m);
  int e = (int)((bits >> 52) & 0x7ff);
  e = (e == 0 || e == 0x7ff) ? 0 : e - 1023;
  e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
  return __builtin_bit_cast(double, (long long)(1023 - e) << 52);
}

// 1/b = conj(b) / (Re b^2 + Im b^2), with b first scaled by an exact power of two s near
// 1/|b| so that the squares neither overflow nor push lower components below the
// normal range: 1/b = s * (1/(s b)).  Every step is exact under scaling by a power of two
// while nothing over- or underflows, so for moderate |b| the result is bit for bit that of
// the unscaled formula.
template <int C>
__host__ __device__ __forceinline__ void zrecip(const double (&br_)[C], const double (&bi_)[C],
                                       double (&or_)[C], double (&oi)[C]) {
  const double s = recip_scale(br_[0], bi_[0]);
  double br[C], bi[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    br[k] = br_[k] * s;
    bi[k] = bi_[k] * s;
  }
  double l[C];
  set_zero<C>(l);
  mac<C>(l, br, br);
  mac<C>(l, bi, bi);
  double d[C], inv[C];
  renorm<C>(l, d);
  recip<C>(d, inv);
  double nbi[C];
  neg<C>(bi, nbi);
  mul<C>(br, inv, or_);
  mul<C>(nbi, inv, oi);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    or_[k] *= s;
    oi[k] *= s;
  }
}

// cabs1 = |Re| + |Im| in full precision
template <int C>
__host__ __device__ __forceinline__ void cabs1(const double (&ar)[C], const double (&ai)[C], double (&o)[C]) {
  double x[C], y[C];
  abs_<C>(ar, x);
  abs_<C>(ai, y);
  add<C>(x, y, o);
}

}  // namespace mp
