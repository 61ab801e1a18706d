// Double-precision complex arithmetic for the device code.
#pragma once

#include <hip/hip_runtime.h>

namespace shgb {

struct cd {
  double re, im;
};

__host__ __device__ inline cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }

// a / b with scaling by the larger component of b (Smith's method).
__host__ __device__ inline cd cdiv(cd a, cd b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, den = b.re + b.im * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  const double r = b.re / b.im, den = b.im + b.re * r;
  return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}

// principal square root (branch cut on the negative real axis)
__host__ __device__ inline cd csqrt_principal(cd z) {
  const double r = hypot(z.re, z.im);
  if (r == 0.0) return {0.0, 0.0};
  if (z.re >= 0.0) {
    const double t = sqrt(0.5 * (r + z.re));
    return {t, z.im / (2.0 * t)};
  }
  const double t = sqrt(0.5 * (r - z.re));
  return {fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

__host__ __device__ inline cd cexp(cd z) {
  double s, c;
  sincos(z.im, &s, &c);
  const double e = exp(z.re);
  return {e * c, e * s};
}

}  // namespace shgb
