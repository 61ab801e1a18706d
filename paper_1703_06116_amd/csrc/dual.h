// Dual numbers (a value and its derivative along one direction) for the
// tangent kernels, and the two-level quantities of the QCLE on them.
#pragma once

#include "cplx.h"
#include "device.h"

namespace shgb {

// value and derivative along one direction
struct Du {
  double v, d;
  Du() = default;
  __host__ __device__ constexpr Du(double x) : v(x), d(0.0) {}
  __host__ __device__ constexpr Du(double x, double dx) : v(x), d(dx) {}
};

__device__ inline Du operator+(Du a, Du b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Du operator-(Du a, Du b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Du operator-(Du a) { return {-a.v, -a.d}; }
__device__ inline Du &operator+=(Du &a, Du b) { return a = a + b; }
__device__ inline Du &operator-=(Du &a, Du b) { return a = a - b; }
__device__ inline Du operator*(Du a, Du b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline Du operator*(double s, Du a) { return {s * a.v, s * a.d}; }
__device__ inline Du operator*(Du a, double s) { return {a.v * s, a.d * s}; }
__device__ inline Du operator/(Du a, Du b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ inline Du dexp(Du a) {
  const double e = exp(a.v);
  return {e, e * a.d};
}
__device__ inline Du dfabs(Du a) { return a.v < 0.0 ? -a : a; }
// |a| with the sign of s (value), as copysign
__device__ inline Du dcopysign(Du a, Du s) {
  const bool neg = (a.v < 0.0) != (s.v < 0.0 || (s.v == 0.0 && signbit(s.v)));
  return neg ? -a : a;
}
__device__ inline Du drecip(Du a) {
  const double r = recip(a.v);
  return {r, -r * r * a.d};
}
__device__ inline Du drsqrt(Du a) {
  const double r = rsqrt_nr(a.v);
  return {r, -0.5 * r * r * r * a.d};
}
__device__ inline Du cst(double v) { return {v, 0.0}; }

struct QcleDu {
  Du A, B, C, D;
  double inv_mass;
};

struct Q1Du {
  Du s, s1, s2, s3, d21;
};

// The two-level quantities of Sec. 3.3 the adiabatic energies and d21 below eq:QCLE and their q-derivatives,
// the same formulas as the FP64 stepping kernel, on (value, derivative) pairs.
__device__ inline Q1Du qcle_q1_du(const QcleDu &p, Du q) {
  const Du x = p.B * q;
  const Du e = dexp(-2.0 * dfabs(x));
  const Du r = drecip(cst(1.0) + e);
  const Du th = dcopysign((cst(1.0) - e) * r, x);
  const Du sech2 = 4.0 * e * r * r;
  const Du AB = p.A * p.B;
  const Du a = p.A * th;
  const Du a1 = AB * sech2;
  const Du a2 = -2.0 * AB * p.B * th * sech2;
  const Du a3 = -2.0 * AB * p.B * p.B * sech2 * (cst(1.0) - 3.0 * th * th);
  const Du q2 = q * q;
  const Du c = p.C * dexp(-(p.D * q2));
  const Du c1 = -2.0 * p.D * q * c;
  const Du c2 = (4.0 * p.D * p.D * q2 - 2.0 * p.D) * c;
  const Du c3 = q * (12.0 * p.D * p.D - 8.0 * p.D * p.D * p.D * q2) * c;
  const Du ss = a * a + c * c;
  const Du rs = drsqrt(ss);
  Q1Du o;
  o.s = ss * rs;
  o.s1 = (a * a1 + c * c1) * rs;
  o.s2 = ((a1 * a1 + a * a2) + (c1 * c1 + c * c2) - o.s1 * o.s1) * rs;
  o.s3 = (3.0 * (a1 * a2 + c1 * c2) + (a * a3 + c * c3) - 3.0 * o.s1 * o.s2) * rs;
  o.d21 = 0.5 * (a * c1 - c * a1) * rs * rs;
  return o;
}

// Hop state of a beam in a tangent pass: the discrete part as in the
// stepping kernels, the weight log w as a dual number.
struct HopDu {
  HopScalars h;  // discrete part (component, hop count, phase sign, threshold); h.logw, h.Lam unused
  Du logw;
  bool pending;
  uint64_t gid, seed;
};

// complex (value, derivative) pairs for the beam integral
struct Cdu {
  cd v, d;
};

__device__ inline Cdu cd_mul(Cdu a, Cdu b) { return {cmul(a.v, b.v), cadd(cmul(a.d, b.v), cmul(a.v, b.d))}; }
__device__ inline Cdu cd_div(Cdu a, Cdu b) {
  const cd q = cdiv(a.v, b.v);
  return {q, cdiv(csub(a.d, cmul(q, b.d)), b.v)};
}
__device__ inline Cdu cd_sqrt(Cdu z) {
  const cd s = csqrt_principal(z.v);
  return {s, cdiv(z.d, cscale(s, 2.0))};
}
__device__ inline Cdu cd_exp(Cdu z) {
  const cd e = cexp(z.v);
  return {e, cmul(e, z.d)};
}
__device__ inline Cdu cd_real(Du x) { return {{x.v, 0.0}, {x.d, 0.0}}; }
__device__ inline Cdu cd_of(Du re, Du im) { return {{re.v, im.v}, {re.d, im.d}}; }

// Per component: sum Re c, sum Im c, d sum Re c, d sum Im c.
constexpr int kTanVals = SHGB_NCOMP * 4;

}  // namespace shgb
