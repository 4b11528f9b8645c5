// Value types for the ML(n)BiCGStab kernels: real and complex, fp64 and fp32.
//
// V  : the type vectors and matrix values are stored in (double, float,
//      cplx<double>, cplx<float>).
// Sc : the type the coefficient recurrences run in; always fp64
//      (double or cplx<double>), also when vectors are fp32.
// u^H v = sum conj(u_i) v_i throughout.
#pragma once

#include <hip/hip_runtime.h>

namespace mlb {

template <class R>
struct cplx {
  R re, im;
};

template <class T> struct traits;
template <> struct traits<double> {
  using real = double;
  using wide = double;            // fp64 counterpart
  static constexpr bool is_complex = false;
};
template <> struct traits<float> {
  using real = float;
  using wide = double;
  static constexpr bool is_complex = false;
};
template <> struct traits<cplx<double>> {
  using real = double;
  using wide = cplx<double>;
  static constexpr bool is_complex = true;
};
template <> struct traits<cplx<float>> {
  using real = float;
  using wide = cplx<double>;
  static constexpr bool is_complex = true;
};

// ---- arithmetic -----------------------------------------------------------

__host__ __device__ inline double conj(double a) { return a; }
__host__ __device__ inline float conj(float a) { return a; }
template <class R>
__host__ __device__ inline cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }

template <class R>
__host__ __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__host__ __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__host__ __device__ inline cplx<R> operator-(cplx<R> a) { return {-a.re, -a.im}; }
template <class R>
__host__ __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__host__ __device__ inline cplx<R> operator*(R s, cplx<R> b) { return {s * b.re, s * b.im}; }
template <class R>
__host__ __device__ inline cplx<R>& operator+=(cplx<R>& a, cplx<R> b) { a.re += b.re; a.im += b.im; return a; }
template <class R>
__host__ __device__ inline bool operator==(cplx<R> a, R b) { return a.re == b && a.im == 0; }

// a / b for complex: scaled by the larger component of b (Smith's method)
template <class R>
__host__ __device__ inline cplx<R> operator/(cplx<R> a, cplx<R> b) {
  R ar = b.re < 0 ? -b.re : b.re;
  R ai = b.im < 0 ? -b.im : b.im;
  if (ar >= ai) {
    R t = b.im / b.re, den = b.re + b.im * t;
    return {(a.re + a.im * t) / den, (a.im - a.re * t) / den};
  } else {
    R t = b.re / b.im, den = b.re * t + b.im;
    return {(a.re * t + a.im) / den, (a.im * t - a.re) / den};
  }
}
template <class R>
__host__ __device__ inline cplx<R> operator/(cplx<R> a, R s) { return {a.re / s, a.im / s}; }

__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline float abs2(float a) { return a * a; }
template <class R>
__host__ __device__ inline R abs2(cplx<R> a) { return a.re * a.re + a.im * a.im; }

__host__ __device__ inline double re(double a) { return a; }
__host__ __device__ inline double re(float a) { return a; }
template <class R>
__host__ __device__ inline R re(cplx<R> a) { return a.re; }

// conj(a) * b accumulated into acc
__device__ inline void cdot_acc(double& acc, double a, double b) { acc = fma(a, b, acc); }
__device__ inline void cdot_acc(float& acc, float a, float b) { acc = fmaf(a, b, acc); }
template <class R>
__device__ inline void cdot_acc(cplx<R>& acc, cplx<R> a, cplx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}

// y + a * x
__device__ inline double axpy(double y, double a, double x) { return fma(a, x, y); }
__device__ inline float axpy(float y, float a, float x) { return fmaf(a, x, y); }
template <class R>
__device__ inline cplx<R> axpy(cplx<R> y, cplx<R> a, cplx<R> x) {
  cplx<R> o;
  o.re = fma(a.re, x.re, y.re);
  o.re = fma(-a.im, x.im, o.re);
  o.im = fma(a.re, x.im, y.im);
  o.im = fma(a.im, x.re, o.im);
  return o;
}

// ---- conversions ----------------------------------------------------------

template <class To, class From> __host__ __device__ inline To convert(From v);
template <> __host__ __device__ inline double convert<double, double>(double v) { return v; }
template <> __host__ __device__ inline float convert<float, double>(double v) { return (float)v; }
template <> __host__ __device__ inline double convert<double, float>(float v) { return (double)v; }
template <> __host__ __device__ inline float convert<float, float>(float v) { return v; }
template <> __host__ __device__ inline cplx<double> convert<cplx<double>, cplx<double>>(cplx<double> v) { return v; }
template <> __host__ __device__ inline cplx<float> convert<cplx<float>, cplx<double>>(cplx<double> v) {
  return {(float)v.re, (float)v.im};
}
template <> __host__ __device__ inline cplx<double> convert<cplx<double>, cplx<float>>(cplx<float> v) {
  return {(double)v.re, (double)v.im};
}
template <> __host__ __device__ inline cplx<float> convert<cplx<float>, cplx<float>>(cplx<float> v) { return v; }

template <class T> __host__ __device__ inline T zero() { return T{}; }
template <class T> __host__ __device__ inline T from_real(double v);
template <> __host__ __device__ inline double from_real<double>(double v) { return v; }
template <> __host__ __device__ inline float from_real<float>(double v) { return (float)v; }
template <> __host__ __device__ inline cplx<double> from_real<cplx<double>>(double v) { return {v, 0.0}; }
template <> __host__ __device__ inline cplx<float> from_real<cplx<float>>(double v) { return {(float)v, 0.f}; }

__host__ __device__ inline bool finite(double a) { return a - a == 0.0; }
template <class R>
__host__ __device__ inline bool finite(cplx<R> a) { return finite((double)a.re) && finite((double)a.im); }
__host__ __device__ inline bool is_zero(double a) { return a == 0.0; }
template <class R>
__host__ __device__ inline bool is_zero(cplx<R> a) { return a.re == 0 && a.im == 0; }

}  // namespace mlb
