// Scalar types shared by host and device code: real double and a plain
// complex double (interleaved re, im).  Complex-symmetric plans use plain
// transposes; Hermitian plans conjugate wherever a transpose appears, through
// cj(v, cs) with cs = -1 (cs = +1 leaves v as it is).  Division uses Smith's algorithm (R. L. Smith,
// "Algorithm 116: Complex division", CACM 5(8), 1962) to avoid overflow.
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define SELINV_HD __host__ __device__ __forceinline__
#else
#define SELINV_HD inline
#endif

namespace selinv {

struct cplx {
  double re, im;
};

SELINV_HD cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
SELINV_HD cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
SELINV_HD cplx operator-(cplx a) { return {-a.re, -a.im}; }
SELINV_HD cplx operator*(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
SELINV_HD cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
SELINV_HD cplx &operator+=(cplx &a, cplx b) { a.re += b.re; a.im += b.im; return a; }
SELINV_HD cplx &operator-=(cplx &a, cplx b) { a.re -= b.re; a.im -= b.im; return a; }

// v for cs = +1, conj(v) for cs = -1 (a Hermitian plan); real values pass through
SELINV_HD double cj(double v, double) { return v; }
SELINV_HD cplx cj(cplx v, double cs) { return {v.re, cs * v.im}; }

SELINV_HD cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  double ar = b.re < 0 ? -b.re : b.re, ai = b.im < 0 ? -b.im : b.im;
  if (ar >= ai) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  } else {
    double r = b.re / b.im, den = b.re * r + b.im;
    return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
  }
}

template <typename T> struct SOps;

template <> struct SOps<double> {
  static SELINV_HD double zero() { return 0.0; }
  static SELINV_HD double one() { return 1.0; }
  static SELINV_HD double div(double a, double b) { return a / b; }
  static SELINV_HD double scale(double s, double a) { return s * a; }
};

template <> struct SOps<cplx> {
  static SELINV_HD cplx zero() { return {0.0, 0.0}; }
  static SELINV_HD cplx one() { return {1.0, 0.0}; }
  static SELINV_HD cplx div(cplx a, cplx b) { return cdiv(a, b); }
  static SELINV_HD cplx scale(double s, cplx a) { return {s * a.re, s * a.im}; }
};

}  // namespace selinv
