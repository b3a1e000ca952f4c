// Host build of the library's multi-component arithmetic (mp.hpp is __host__ __device__)
// so that the CPU test-suite can check it against the oracle without a GPU.
#include "../../paper_2403_16013_amd/csrc/mp.hpp"

template <int C>
static void cp_in(const double *p, double (&v)[C]) {
  for (int k = 0; k < C; ++k) v[k] = p[k];
}
template <int C>
static void cp_out(const double (&v)[C], double *p) {
  for (int k = 0; k < C; ++k) p[k] = v[k];
}

#define DISPATCH(C, ...) \
  switch (C) {            \
    case 2: { constexpr int K = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int K = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int K = 4; __VA_ARGS__; } break; \
  }

extern "C" {

void mph_renorm(int C, const double *a, double *o) {
  DISPATCH(C, { double x[K], y[K]; cp_in<K>(a, x); mp::renorm<K>(x, y); cp_out<K>(y, o); })
}
void mph_add(int C, const double *a, const double *b, double *o) {
  DISPATCH(C, { double x[K], y[K], z[K]; cp_in<K>(a, x); cp_in<K>(b, y); mp::add<K>(x, y, z); cp_out<K>(z, o); })
}
void mph_mul(int C, const double *a, const double *b, double *o) {
  DISPATCH(C, { double x[K], y[K], z[K]; cp_in<K>(a, x); cp_in<K>(b, y); mp::mul<K>(x, y, z); cp_out<K>(z, o); })
}
void mph_recip(int C, const double *a, double *o) {
  DISPATCH(C, { double x[K], z[K]; cp_in<K>(a, x); mp::recip<K>(x, z); cp_out<K>(z, o); })
}
// complex values as [re_0..re_{C-1}, im_0..im_{C-1}]
void mph_zfms(int C, const double *a, const double *l, const double *u, double *o) {
  DISPATCH(C, {
    double ar[K], ai[K], lr[K], li[K], ur[K], ui[K], orr[K], oi[K];
    cp_in<K>(a, ar); cp_in<K>(a + C, ai); cp_in<K>(l, lr); cp_in<K>(l + C, li);
    cp_in<K>(u, ur); cp_in<K>(u + C, ui);
    mp::zfms<K>(ar, ai, lr, li, ur, ui, orr, oi);
    cp_out<K>(orr, o); cp_out<K>(oi, o + C);
  })
}
void mph_zmul(int C, const double *a, const double *b, double *o) {
  DISPATCH(C, {
    double ar[K], ai[K], br[K], bi[K], orr[K], oi[K];
    cp_in<K>(a, ar); cp_in<K>(a + C, ai); cp_in<K>(b, br); cp_in<K>(b + C, bi);
    mp::zmul<K>(ar, ai, br, bi, orr, oi);
    cp_out<K>(orr, o); cp_out<K>(oi, o + C);
  })
}
void mph_zrecip(int C, const double *a, double *o) {
  DISPATCH(C, {
    double ar[K], ai[K], orr[K], oi[K];
    cp_in<K>(a, ar); cp_in<K>(a + C, ai);
    mp::zrecip<K>(ar, ai, orr, oi);
    cp_out<K>(orr, o); cp_out<K>(oi, o + C);
  })
}
// sum_i a_i b_i with the accumulator re-levelled (mp::tidy) after every `period` terms
void mph_dot_tidy(int C, int n, int period, const double *a, const double *b, double *o) {
  DISPATCH(C, {
    double l[K];
    mp::set_zero<K>(l);
    for (int i = 0; i < n; ++i) {
      double x[K], y[K];
      cp_in<K>(a + i * C, x); cp_in<K>(b + i * C, y);
      mp::mac<K>(l, x, y);
      if (period > 0 && (i + 1) % period == 0) mp::tidy<K>(l);
    }
    double z[K];
    mp::renorm<K>(l, z);
    cp_out<K>(z, o);
  })
}
// the raw levels of mp::tidy applied to a C-level accumulator given as l[C]
void mph_tidy(int C, const double *l, double *o) {
  DISPATCH(C, {
    double v[K];
    cp_in<K>(l, v);
    mp::tidy<K>(v);
    cp_out<K>(v, o);
  })
}
// sum_i a_i b_i of n real values (row-major n x C) in one level accumulator
void mph_dot(int C, int n, const double *a, const double *b, double *o) {
  DISPATCH(C, {
    double l[K];
    mp::set_zero<K>(l);
    for (int i = 0; i < n; ++i) {
      double x[K], y[K];
      cp_in<K>(a + i * C, x); cp_in<K>(b + i * C, y);
      mp::mac<K>(l, x, y);
    }
    double z[K];
    mp::renorm<K>(l, z);
    cp_out<K>(z, o);
  })
}
}
