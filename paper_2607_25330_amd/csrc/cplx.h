// Complex arithmetic for the PSFD kernels (interleaved re/im pairs, 8- or 16-byte aligned).
#pragma once
#include <hip/hip_runtime.h>

namespace psfd {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) {
  return cplx<T>{r, i};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a) {
  return {-a.re, -a.im};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) {
  return {s * a.re, s * a.im};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> conj(cplx<T> a) {
  return {a.re, -a.im};
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cplx<T> mul_i(cplx<T> a) {
  return {-a.im, a.re};
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ T norm2(cplx<T> a) {
  return a.re * a.re + a.im * a.im;
}
template <typename U, typename T>
__host__ __device__ __forceinline__ cplx<U> cast(cplx<T> a) {
  return {static_cast<U>(a.re), static_cast<U>(a.im)};
}

// Division by Smith's method (no overflow for large operands).
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
  if (fabs(b.re) >= fabs(b.im)) {
    T r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    T r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}

// Square root on the branch Im >= 0 (Re >= 0 when Im == 0): the outgoing or
// decaying axial wavenumber for the time factor exp(-i omega t).
__host__ __device__ inline cplx<double> sqrt_up(cplx<double> w) {
  double x = w.re, y = w.im;
  double r = hypot(x, y);
  double t = sqrt(0.5 * (r + fabs(x)));
  cplx<double> q;
  if (t == 0.0) {
    q = {0.0, 0.0};
  } else if (x >= 0.0) {
    q = {t, y / (2.0 * t)};
  } else {
    q = {fabs(y) / (2.0 * t), copysign(t, y)};
  }
  if (q.im < 0.0 || (q.im == 0.0 && q.re < 0.0)) q = {-q.re, -q.im};
  return q;
}

__device__ __forceinline__ void sc(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sc(double x, double* s, double* c) { sincos(x, s, c); }

// exp(i w) for complex w.
__host__ __device__ inline cplx<double> cexpi(cplx<double> w) {
  double s, c;
  sincos(w.re, &s, &c);
  double m = exp(-w.im);
  return {m * c, m * s};
}

__host__ __device__ inline cplx<double> ccos(cplx<double> w) {
  double s, c;
  sincos(w.re, &s, &c);
  return {c * cosh(w.im), -s * sinh(w.im)};
}
__host__ __device__ inline cplx<double> csin(cplx<double> w) {
  double s, c;
  sincos(w.re, &s, &c);
  return {s * cosh(w.im), c * sinh(w.im)};
}

}  // namespace psfd
