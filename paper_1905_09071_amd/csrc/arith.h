// Device arithmetic for the three spectral precisions of the library:
//   double  - binary64 throughout
//   float   - binary32 spectra, twiddles rounded from binary64
//   ff      - float-float pairs (hi + lo) carried through the whole spectral
//             path with error-free transforms (TwoSum, Fast2Sum, FMA-based
//             TwoProd); about 44 significant bits at binary32 storage width x2.
// The state vector, the loss-term dot products and all moment sums stay in
// binary64 in every mode.
//
// Build note: everything here relies on IEEE round-to-nearest, no flush of
// binary32 subnormals, and no reassociation (never compile with fast-math).
// The library is built with -ffp-contract=off: a multiply and an add are fused
// only where the source says so (__builtin_fma).  Besides keeping the
// float-float error-free transforms exact (fusing TwoProd's rounded product
// with a following Fast2Sum would destroy the error terms), this makes every
// expression round the same way in every kernel variant that inlines it.
#pragma once
#include <hip/hip_runtime.h>

struct ff {
  float hi, lo;
};

// ---- error-free transforms -------------------------------------------------
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void fast_two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  e = b - (s - a);
}

// Dekker's addition without the final renormalisation: the error term of the
// two high parts is kept exactly and the low parts are added once, so
// |result - (a+b)| <= ~2^-46 (|a| + |b|).  The pair it returns is not
// renormalised (|lo| may exceed half an ulp of hi by a small factor); every
// value that leaves registers (LDS, global memory) goes through ff_norm, which
// bounds the growth of lo to the few operations between two stores.  The
// absolute bound is what the normwise error of a transform, a product of
// spectra and an inverse transform depends on; relative accuracy under
// cancellation is not needed here.
__device__ __forceinline__ ff operator+(ff a, ff b) {
#pragma clang fp contract(off)
  float s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  return ff{s, e};
}
__device__ __forceinline__ ff operator-(ff a) { return ff{-a.hi, -a.lo}; }
__device__ __forceinline__ ff operator-(ff a, ff b) { return a + (-b); }
// Exact product of the high parts (FMA TwoProd) plus the two cross terms; the
// pair is left unrenormalised as for the sum.
__device__ __forceinline__ ff operator*(ff a, ff b) {
#pragma clang fp contract(off)
  float p = a.hi * b.hi;
  float e = __builtin_fmaf(a.hi, b.hi, -p);
  e = __builtin_fmaf(a.hi, b.lo, e);
  e = __builtin_fmaf(a.lo, b.hi, e);
  return ff{p, e};
}
__device__ __forceinline__ ff ff_norm(ff a) {
  ff r;
  fast_two_sum(a.hi, a.lo, r.hi, r.lo);
  return r;
}

// ---- conversions -----------------------------------------------------------
template <class T> struct Real;
template <> struct Real<double> {
  static __device__ __forceinline__ double norm(double x) { return x; }
  static __device__ __forceinline__ double from_d(double x) { return x; }
  static __device__ __forceinline__ double to_d(double x) { return x; }
  static __device__ __forceinline__ double zero() { return 0.0; }
};
template <> struct Real<float> {
  static __device__ __forceinline__ float norm(float x) { return x; }
  static __device__ __forceinline__ float from_d(double x) { return (float)x; }
  static __device__ __forceinline__ double to_d(float x) { return (double)x; }
  static __device__ __forceinline__ float zero() { return 0.0f; }
};
template <> struct Real<ff> {
  static __device__ __forceinline__ ff norm(ff x) { return ff_norm(x); }
  static __device__ __forceinline__ ff from_d(double x) {
    float h = (float)x;
    return ff{h, (float)(x - (double)h)};
  }
  static __device__ __forceinline__ double to_d(ff x) { return (double)x.hi + (double)x.lo; }
  static __device__ __forceinline__ ff zero() { return ff{0.0f, 0.0f}; }
};

// ---- complex ---------------------------------------------------------------
template <class T> struct cplx {
  T re, im;
};

template <class T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return cplx<T>{a.re + b.re, a.im + b.im};
}
template <class T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return cplx<T>{a.re - b.re, a.im - b.im};
}
template <class T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cplx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <class T> __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return cplx<T>{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// Native formats: one product and one fused multiply-add per part, written
// out.  The library is compiled without automatic contraction, so every
// kernel variant rounds a given expression the same way (a state's result
// does not depend on which variant a launch used); the fused forms that matter
// are explicit.
__device__ __forceinline__ cplx<double> cmul(cplx<double> a, cplx<double> b) {
  return cplx<double>{__builtin_fma(a.re, b.re, -(a.im * b.im)), __builtin_fma(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplx<double> cmulc(cplx<double> a, cplx<double> b) {
  return cplx<double>{__builtin_fma(a.re, b.re, a.im * b.im), __builtin_fma(a.im, b.re, -(a.re * b.im))};
}
__device__ __forceinline__ cplx<float> cmul(cplx<float> a, cplx<float> b) {
  return cplx<float>{__builtin_fmaf(a.re, b.re, -(a.im * b.im)), __builtin_fmaf(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplx<float> cmulc(cplx<float> a, cplx<float> b) {
  return cplx<float>{__builtin_fmaf(a.re, b.re, a.im * b.im), __builtin_fmaf(a.im, b.re, -(a.re * b.im))};
}
template <class T> __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return cplx<T>{a.re, -a.im}; }
template <class T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) {
  return cplx<T>{a.re * s, a.im * s};
}
// multiply by +i and by -i
template <class T> __device__ __forceinline__ cplx<T> cmul_i(cplx<T> a) { return cplx<T>{-a.im, a.re}; }
template <class T> __device__ __forceinline__ cplx<T> cmul_negi(cplx<T> a) { return cplx<T>{a.im, -a.re}; }

// renormalised copy (float-float) for storing; identity otherwise
template <class T> __device__ __forceinline__ cplx<T> cnorm(cplx<T> a) {
  return cplx<T>{Real<T>::norm(a.re), Real<T>::norm(a.im)};
}

template <class T> __device__ __forceinline__ cplx<T> czero() {
  return cplx<T>{Real<T>::zero(), Real<T>::zero()};
}

// Halving is exact in every format (barring underflow), so it is a plain scale.
template <class T> __device__ __forceinline__ T half_of(T x);
template <> __device__ __forceinline__ double half_of(double x) { return 0.5 * x; }
template <> __device__ __forceinline__ float half_of(float x) { return 0.5f * x; }
template <> __device__ __forceinline__ ff half_of(ff x) { return ff{0.5f * x.hi, 0.5f * x.lo}; }
