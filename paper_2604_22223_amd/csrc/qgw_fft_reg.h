// In-register mixed-radix (4, 2, 3, 5) DFT of a compile-time length N.
//
// X[q] = sum_s x[s] exp(SIGN * 2 pi i s q / N), natural order in and out.
// Self-sorting (Stockham) passes: with NS the product of the radices done so
// far and P the next radix, butterfly j reads x[j + r N/P] (r < P), applies
// the twiddles exp(SIGN 2 pi i r (j mod NS) / (NS P)), does a P-point DFT and
// writes y[(j / NS) NS P + (j mod NS) + r NS].  All loops unroll fully, so
// every index is a compile-time constant and x lives in registers.
//
// ``tw`` holds exp(-2 pi i e / N) for e = 0 .. N-1; its addresses are uniform
// across a wavefront, so the loads become scalar loads.
#pragma once
#include "qgw_complex.h"

namespace qgw {

constexpr int fft_radix(int n) {
  return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : (n % 5 == 0) ? 5 : n;
}

// exp(SIGN 2 pi i e / N) with the exact values at the quarter turns.
template <int N, int SIGN, typename T>
__host__ __device__ __forceinline__ cpx<T> twiddle_mul(cpx<T> v, const cpx<T>* __restrict__ tw, int e) {
  if (e == 0) return v;
  if (4 * e == N) return mul_i<SIGN>(v);
  if (2 * e == N) return -v;
  if (4 * e == 3 * N) return mul_i<-SIGN>(v);
  cpx<T> w = tw[e];
  if (SIGN > 0) w = conj(w);
  return v * w;
}

template <int P, int SIGN, typename T>
__host__ __device__ __forceinline__ void dft_small(cpx<T> (&v)[P]) {
  if constexpr (P == 2) {
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (P == 4) {
    cpx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
    cpx<T> s13 = v[1] + v[3], d13 = mul_i<SIGN>(v[1] - v[3]);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + d13;
    v[3] = d02 - d13;
  } else if constexpr (P == 3) {
    const T h = T(0.866025403784438646763723170752936183);  // sin(2 pi / 3)
    cpx<T> t1 = v[1] + v[2];
    cpx<T> t2 = scale(mul_i<SIGN>(v[1] - v[2]), h);
    cpx<T> m = v[0] - scale(t1, T(0.5));
    v[0] = v[0] + t1;
    v[1] = m + t2;
    v[2] = m - t2;
  } else if constexpr (P == 5) {
    const T c1 = T(0.309016994374947424102293417182819059);   // cos(2 pi / 5)
    const T c2 = T(-0.809016994374947424102293417182819059);  // cos(4 pi / 5)
    const T s1 = T(0.951056516295153572116439333379382143);   // sin(2 pi / 5)
    const T s2 = T(0.587785252292473129168705954639072769);   // sin(4 pi / 5)
    cpx<T> t1 = v[1] + v[4], t2 = v[2] + v[3];
    cpx<T> t3 = v[1] - v[4], t4 = v[2] - v[3];
    cpx<T> a1 = v[0] + scale(t1, c1) + scale(t2, c2);
    cpx<T> a2 = v[0] + scale(t1, c2) + scale(t2, c1);
    cpx<T> b1 = mul_i<SIGN>(scale(t3, s1) + scale(t4, s2));
    cpx<T> b2 = mul_i<SIGN>(scale(t3, s2) - scale(t4, s1));
    v[0] = v[0] + t1 + t2;
    v[1] = a1 + b1;
    v[4] = a1 - b1;
    v[2] = a2 + b2;
    v[3] = a2 - b2;
  } else {
    static_assert(P == 1, "radix must be 1, 2, 3, 4 or 5");
  }
}

template <int N, int SIGN, int NS, typename T>
__host__ __device__ __forceinline__ void fft_pass(cpx<T> (&x)[N], const cpx<T>* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int P = fft_radix(N / NS);
    static_assert(P <= 5, "mesh side must factor into 2, 3 and 5");
    cpx<T> y[N];
#pragma unroll
    for (int j = 0; j < N / P; ++j) {
      const int k = j % NS;
      cpx<T> v[P];
#pragma unroll
      for (int r = 0; r < P; ++r) v[r] = x[j + r * (N / P)];
#pragma unroll
      for (int r = 1; r < P; ++r) v[r] = twiddle_mul<N, SIGN>(v[r], tw, (r * k * (N / (NS * P))) % N);
      dft_small<P, SIGN>(v);
      const int base = (j / NS) * NS * P + k;
#pragma unroll
      for (int r = 0; r < P; ++r) y[base + r * NS] = v[r];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = y[i];
    fft_pass<N, SIGN, NS * P>(x, tw);
  }
}

template <int N, int SIGN, typename T>
__host__ __device__ __forceinline__ void fft_reg(cpx<T> (&x)[N], const cpx<T>* __restrict__ tw) {
  fft_pass<N, SIGN, 1>(x, tw);
}

}  // namespace qgw

namespace qgw {

// A slab is one N x N mesh (row-major, index = x1 N + x2).  In LDS it is
// stored with a row stride of N + 1 so that strided column reads spread
// over the banks.
template <int N>
struct MeshShape {
  static constexpr int NN = N * N;
  static constexpr int LD = N + 1;
  static constexpr int SLAB = N * LD;  // LDS elements per slab
};

// Logical block of hardware block b in a grid of nb blocks.  The dispatcher deals
// blocks round-robin to the eight XCDs (block b runs on XCD b mod 8), each with
// its own L2; this bijection hands every XCD one contiguous range of logical
// blocks instead, so blocks that read the same G slabs (neighbouring pair slabs,
// or the outputs of one time node) share an L2 and those slabs leave HBM once.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t per = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
  return x * per + (x < rem ? x : rem) + i;
}

// Slab count per block: enough lines for a few waves, LDS-bounded.
template <typename T>
static inline int slabs_per_block(int n, int lds_budget) {
  const int slab_bytes = n * (n + 1) * int(sizeof(cpx<T>));
  int s = 256 / n;
  if (s < 1) s = 1;
  while (s > 1 && s * slab_bytes > lds_budget) --s;
  return s;
}

}  // namespace qgw
