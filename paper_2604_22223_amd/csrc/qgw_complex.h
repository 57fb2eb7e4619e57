// Complex arithmetic shared by the libqgw kernels (device and host).
#pragma once
#include <hip/hip_runtime.h>

namespace qgw {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

using zd = cpx<double>;
using zf = cpx<float>;

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T re, T im) {
  cpx<T> z;
  z.re = re;
  z.im = im;
  return z;
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return mk(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return mk(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a) {
  return mk(-a.re, -a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) {
  return mk(a.re * s, a.im * s);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) {
  return mk(a.re, -a.im);
}
// a + b * c
template <typename T>
__host__ __device__ __forceinline__ cpx<T> fma(cpx<T> a, cpx<T> b, cpx<T> c) {
  return mk(a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re);
}
// a - b * c
template <typename T>
__host__ __device__ __forceinline__ cpx<T> fms(cpx<T> a, cpx<T> b, cpx<T> c) {
  return mk(a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re);
}
// i * s * a  (s = +1 or -1)
template <int S, typename T>
__host__ __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
  return S > 0 ? mk(-a.im, a.re) : mk(a.im, -a.re);
}
template <typename T>
__host__ __device__ __forceinline__ T norm2(cpx<T> a) {
  return a.re * a.re + a.im * a.im;
}
// x if finite, else +inf: a max-reduction through fmax then keeps NaNs visible
__host__ __device__ __forceinline__ double finite_or_inf(double x) { return __builtin_isfinite(x) ? x : INFINITY; }
// 1 / a
template <typename T>
__host__ __device__ __forceinline__ cpx<T> inv(cpx<T> a) {
  T d = T(1) / norm2(a);
  return mk(a.re * d, -a.im * d);
}

template <typename T, typename U>
__host__ __device__ __forceinline__ cpx<T> cast(cpx<U> a) {
  return mk(static_cast<T>(a.re), static_cast<T>(a.im));
}

}  // namespace qgw
