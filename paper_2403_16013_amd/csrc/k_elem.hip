// k_elem.hip -- element-wise kernels: canonicalisation of stored components, precision
// conversion, integer fill, and the row permutation used by the solves.
#include "common.hpp"

#pragma clang fp contract(off)

namespace mplu {

template <int C>
__global__ __launch_bounds__(256) void k_renorm(int64_t m, int64_t n, ZM A) {
  const int64_t total = m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % m, j = e / m;
    double re[C], im[C], o[C];
    ld_z<C>(A, i, j, re, im);
    mp::renorm<C>(re, o);
    mp::copy<C>(o, re);
    mp::renorm<C>(im, o);
    st_z<C>(A, i, j, re, o);
  }
}

// Cs -> Cd components.  Widening copies and zero-pads (exact).  Narrowing renormalises,
// then folds the dropped tail into the last kept component.
template <int Cs, int Cd>
__global__ __launch_bounds__(256) void k_convert(int64_t m, int64_t n, ZM A, ZM B) {
  const int64_t total = m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % m, j = e / m;
    double re[Cs], im[Cs];
    ld_z<Cs>(A, i, j, re, im);
    double part[2][Cs];
    mp::renorm<Cs>(re, part[0]);
    mp::renorm<Cs>(im, part[1]);
    double o[2][Cd];
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
#pragma unroll
      for (int c = 0; c < Cd; ++c) o[ri][c] = c < Cs ? part[ri][c] : 0.0;
      if (Cd < Cs) {
        double tail = 0.0;
#pragma unroll
        for (int c = Cs - 1; c >= Cd; --c) tail += part[ri][c];
        o[ri][Cd - 1] += tail;
      }
    }
    st_z<Cd>(B, i, j, o[0], o[1]);
  }
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// perm[k] = original row that ends up at row k after the interchanges of ipiv, applied in
// order (one workgroup: the row index array lives in LDS while the swaps are replayed).
// perm[i] = the original row that the interchanges ipiv[0..n) (applied in order, LAPACK
// laswp semantics) bring to position i.  The interchange sequence is inherently serial,
// but each original row's path through it is independent: thread r follows row r's
// position through all n interchanges (ipiv staged in LDS in chunks, read by broadcast)
// and finally records perm[position] = r.
static constexpr int PERM_CHUNK = 8192;

__global__ __launch_bounds__(1024) void k_perm(const int32_t *ipiv, int64_t n, int32_t *perm) {
  __shared__ int32_t sp[PERM_CHUNK];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t pos = r;
  for (int64_t k0 = 0; k0 < n; k0 += PERM_CHUNK) {
    const int cnt = (int)((n - k0) < PERM_CHUNK ? (n - k0) : PERM_CHUNK);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) sp[i] = ipiv[k0 + i] - 1;
    __syncthreads();
    for (int i = 0; i < cnt; ++i) {
      const int64_t k = k0 + i;
      int64_t p = sp[i];
      if (p < 0 || p >= n) p = k;  // an invalid entry swaps nothing
      pos = (pos == k) ? p : ((pos == p) ? k : pos);
    }
  }
  if (r < n) perm[pos] = (int32_t)r;
}

// gather: W[k, :] = B[perm[k], :];  scatter: B[perm[k], :] = W[k, :]  (over `planes`
// planes: 2C for complex, C for real matrices)
__global__ __launch_bounds__(256) void k_gather(const int32_t *perm, int64_t n, int64_t nrhs,
                                                ZM B, ZM W, int scatter, int planes) {
  const int64_t total = n * nrhs * planes;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e % n;
    const int64_t rest = e / n;
    const int64_t r = rest % nrhs;
    const int64_t q = rest / nrhs;
    const int64_t src = perm ? perm[k] : k;
    double *bp = B.p + q * B.ps + r * B.ld + src;
    double *wp = W.p + q * W.ps + r * W.ld + k;
    if (scatter) *bp = *wp;
    else *wp = *bp;
  }
}

// O := sa A + sb B for complex matrices (sa, sb in {-1, 0, 1}; a zero coefficient drops
// the term), one rounding per part; O may be A or B (each element is read before it is
// written by the same thread).  The matrix sums of Winograd's variant of Strassen's
// algorithm and the final C := beta C + alpha W.
template <int C>
__global__ __launch_bounds__(256) void k_zaxpby(int64_t m, int64_t n, int sa, ZM A, int sb, ZM B,
                                                ZM O) {
  const int64_t total = m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % m, j = e / m;
    double lr[C], li[C];
    mp::set_zero<C>(lr);
    mp::set_zero<C>(li);
    double xr[C], xi[C];
    if (sa != 0) {
      ld_z<C>(A, i, j, xr, xi);
      if (sa > 0) { mp::push_mp<C>(lr, xr); mp::push_mp<C>(li, xi); }
      else { mp::push_mp_neg<C>(lr, xr); mp::push_mp_neg<C>(li, xi); }
    }
    if (sb != 0) {
      ld_z<C>(B, i, j, xr, xi);
      if (sb > 0) { mp::push_mp<C>(lr, xr); mp::push_mp<C>(li, xi); }
      else { mp::push_mp_neg<C>(lr, xr); mp::push_mp_neg<C>(li, xi); }
    }
    double orr[C], oi[C];
    mp::renorm<C>(lr, orr);
    mp::renorm<C>(li, oi);
    st_z<C>(O, i, j, orr, oi);
  }
}

static inline int grid_for(int64_t total, int threads) {
  int64_t g = (total + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_renorm(int C, int64_t m, int64_t n, ZM A, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int g = grid_for(m * n, 256);
  switch (C) {
    case 2: hipLaunchKernelGGL(k_renorm<2>, dim3(g), dim3(256), 0, s, m, n, A); break;
    case 3: hipLaunchKernelGGL(k_renorm<3>, dim3(g), dim3(256), 0, s, m, n, A); break;
    case 4: hipLaunchKernelGGL(k_renorm<4>, dim3(g), dim3(256), 0, s, m, n, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define CONV_CASE(a, b)                                                               \
  if (Cs == a && Cd == b) {                                                           \
    hipLaunchKernelGGL((k_convert<a, b>), dim3(g), dim3(256), 0, s, m, n, A, B);      \
    return hipGetLastError();                                                         \
  }

hipError_t launch_convert(int Cs, int Cd, int64_t m, int64_t n, ZM A, ZM B, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int g = grid_for(m * n, 256);
  CONV_CASE(2, 2) CONV_CASE(2, 3) CONV_CASE(2, 4)
  CONV_CASE(3, 2) CONV_CASE(3, 3) CONV_CASE(3, 4)
  CONV_CASE(4, 2) CONV_CASE(4, 3) CONV_CASE(4, 4)
  return hipErrorInvalidValue;
}

hipError_t launch_zaxpby(int C, int64_t m, int64_t n, int sa, ZM A, int sb, ZM B, ZM O,
                         hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int g = grid_for(m * n, 256);
  switch (C) {
    case 2: hipLaunchKernelGGL(k_zaxpby<2>, dim3(g), dim3(256), 0, s, m, n, sa, A, sb, B, O); break;
    case 3: hipLaunchKernelGGL(k_zaxpby<3>, dim3(g), dim3(256), 0, s, m, n, sa, A, sb, B, O); break;
    case 4: hipLaunchKernelGGL(k_zaxpby<4>, dim3(g), dim3(256), 0, s, m, n, sa, A, sb, B, O); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, 256)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_perm(const int32_t *ipiv, int64_t n, int32_t *perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_perm, dim3((unsigned)((n + 1023) / 1024)), dim3(1024), 0, s, ipiv, n, perm);
  return hipGetLastError();
}

hipError_t launch_gather_rows(int C, const int32_t *perm, int64_t n, int64_t nrhs, ZM B, ZM W,
                              bool scatter, hipStream_t s, bool real) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (C < 2 || C > 4) return hipErrorInvalidValue;
  const int planes = real ? C : 2 * C;
  const int g = grid_for(n * nrhs * planes, 256);
  hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, s, perm, n, nrhs, B, W, (int)scatter,
                     planes);
  return hipGetLastError();
}

}  // namespace mplu
