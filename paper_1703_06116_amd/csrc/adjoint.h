// Building blocks of the reverse-mode (adjoint) derivative of the
// populations: the Jacobian of the QCLE two-level quantities with respect to
// q1 and the potential parameters, the leg structure of one interval of the
// hop algorithm, and the checkpoint layout shared by the forward entry point
// and the reverse kernels.
//
// The derivative is that of the discrete algorithm with its events frozen
// (the same one the tangent kernels propagate forwards): every hop test,
// destination and phase sign is decided by the values, the drawn thresholds
// carry no derivative, and a hop time moves with the state through
// theta = (E - Lam)/(Lam' - Lam) (Sec. 2.4 step 4) and the shortened step it
// sets.  Adjoint variables of the packed Hessian entries are the partial
// derivatives with respect to the packed (stored) variables.
#pragma once

#include "cplx.h"
#include "device.h"

namespace shgb {

// A value and its partial derivatives along (q1, A, B, C, D).
constexpr int kJ5 = 5;
struct D5 {
  double v, d[kJ5];
};

__host__ __device__ inline D5 d5c(double x) {
  D5 r;
  r.v = x;
  for (int i = 0; i < kJ5; ++i) r.d[i] = 0.0;
  return r;
}
__host__ __device__ inline D5 d5var(double x, int i) {
  D5 r = d5c(x);
  r.d[i] = 1.0;
  return r;
}
__host__ __device__ inline D5 operator+(const D5 &a, const D5 &b) {
  D5 r;
  r.v = a.v + b.v;
  for (int i = 0; i < kJ5; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
__host__ __device__ inline D5 operator-(const D5 &a, const D5 &b) {
  D5 r;
  r.v = a.v - b.v;
  for (int i = 0; i < kJ5; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
__host__ __device__ inline D5 operator-(const D5 &a) {
  D5 r;
  r.v = -a.v;
  for (int i = 0; i < kJ5; ++i) r.d[i] = -a.d[i];
  return r;
}
__host__ __device__ inline D5 operator*(const D5 &a, const D5 &b) {
  D5 r;
  r.v = a.v * b.v;
  for (int i = 0; i < kJ5; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
__host__ __device__ inline D5 operator*(double s, const D5 &a) {
  D5 r;
  r.v = s * a.v;
  for (int i = 0; i < kJ5; ++i) r.d[i] = s * a.d[i];
  return r;
}
// f(a) with f(a.v) = fv and f'(a.v) = fd
__host__ __device__ inline D5 d5chain(const D5 &a, double fv, double fd) {
  D5 r;
  r.v = fv;
  for (int i = 0; i < kJ5; ++i) r.d[i] = fd * a.d[i];
  return r;
}
__host__ __device__ inline D5 d5exp(const D5 &a) {
  const double e = exp(a.v);
  return d5chain(a, e, e);
}
__host__ __device__ inline D5 d5recip(const D5 &a) {
  const double r = 1.0 / a.v;
  return d5chain(a, r, -r * r);
}
__host__ __device__ inline D5 d5rsqrt(const D5 &a) {
  const double r = 1.0 / sqrt(a.v);
  return d5chain(a, r, -0.5 * r * r * r);
}
__host__ __device__ inline D5 d5abs(const D5 &a) { return a.v < 0.0 ? -a : a; }

// The two-level quantities (s, s', s'', s''', d21) of Sec. 3.3 (the adiabatic
// energies and d21 below eq:QCLE) as functions of (q1, A, B, C, D):
// out[o] for o = s, s1, s2, s3, d21.  The formulas are those of qcle_q1,
// differentiated by the chain rule; only the partials are used.
__host__ __device__ inline void qcle_q1_d5(const DevModel &md, double q1, D5 out[5]) {
  const D5 q = d5var(q1, 0), A = d5var(md.A, 1), B = d5var(md.B, 2), C = d5var(md.C, 3), D = d5var(md.D, 4);
  const D5 x = B * q;
  const D5 e = d5exp(-2.0 * d5abs(x));
  const D5 r = d5recip(d5c(1.0) + e);
  D5 th = (d5c(1.0) - e) * r;
  if (x.v < 0.0) th = -th;
  const D5 sech2 = 4.0 * (e * r * r);
  const D5 AB = A * B;
  const D5 a = A * th;
  const D5 a1 = AB * sech2;
  const D5 a2 = -2.0 * (AB * B * th * sech2);
  const D5 a3 = -2.0 * (AB * B * B * sech2 * (d5c(1.0) - 3.0 * (th * th)));
  const D5 qq = q * q;
  const D5 c = C * d5exp(-(D * qq));
  const D5 c1 = -2.0 * (D * q * c);
  const D5 c2 = (4.0 * (D * D * qq) - 2.0 * D) * c;
  const D5 c3 = q * (12.0 * (D * D) - 8.0 * (D * D * D * qq)) * c;
  const D5 ss = a * a + c * c;
  const D5 rs = d5rsqrt(ss);
  out[0] = ss * rs;
  out[1] = (a * a1 + c * c1) * rs;
  out[2] = ((a1 * a1 + a * a2) + (c1 * c1 + c * c2) - out[1] * out[1]) * rs;
  out[3] = (3.0 * (a1 * a2 + c1 * c2) + (a * a3 + c * c3) - 3.0 * (out[1] * out[2])) * rs;
  out[4] = 0.5 * ((a * c1 - c * a1) * rs * rs);
}

// Adjoints (sb[o], o = s, s1, s2, s3, d21) of the two-level quantities
// pulled back to q1 (returned) and to (A, B, C, D) (added to th[0..3]).
__host__ __device__ inline double q1_pullback(const DevModel &md, double q1, const double sb[5], double th[4]) {
  D5 o[5];
  qcle_q1_d5(md, q1, o);
  double qb = 0.0;
  for (int k = 0; k < 5; ++k) {
    qb += sb[k] * o[k].d[0];
    for (int j = 0; j < 4; ++j) th[j] += sb[k] * o[k].d[1 + j];
  }
  return qb;
}

// Interval legs (Sec. 2.4 steps 3-5).  An interval is run as legs: a leg
// starts at a state y on component l with rem of the interval left, takes
// the trial step y' = Phi_rem(y), and either ends the interval (no hop:
// y' is the result) or hops at the interpolated time (the shortened step
// Phi_{theta rem}(y), then the weight update logw += Lam, Lam = 0, and the
// next leg with rem (1 - theta) on the new component).
enum LegKind : int { kLegAccept = 0, kLegPartial = 1, kLegEnd = 2, kLegNow = 3 };

// Per-block partial sums of the reverse kernels: dA, dB, dC, dD, dp_mean, the
// objective, two unused.
constexpr int kAdjVals = 8;

// ---------------------------------------------------------------------------
// Checkpoints: every `every` intervals the whole state of every beam, in the
// state layout with ld = n (the FP64 rows, then comp and nhop as int32).
struct CkptLayout {
  int64_t n, rows, stride_bytes;  // one checkpoint
  int n_ckpt;
};

__host__ __device__ inline CkptLayout ckpt_layout(int64_t n, int m, int nsteps, int every) {
  CkptLayout c;
  c.n = n;
  c.rows = shgb_nfields(m);
  const int64_t bytes = c.rows * n * 8 + 2 * n * 4;
  c.stride_bytes = (bytes + 255) / 256 * 256;
  c.n_ckpt = (nsteps + every - 1) / every;
  return c;
}

}  // namespace shgb
