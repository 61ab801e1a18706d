// Reverse-mode derivative of the populations of the one-dimensional QCLE
// (phase space m = 2): the per-beam arithmetic, for the device kernel and
// for host builds.  One interval's forward run (the same arithmetic as the
// FP64 stepping kernel, with a hop completed where it starts, at the same
// state) and its reverse sweep through the legs of adjoint.h.
#pragma once

#include "adjoint.h"

namespace shgb {

// The integrated quantities of one beam (m = 2), in the order of the
// stepping kernel.
struct A2 {
  double q, p, Pq, Pp, zr11, zr12, zr22, zi11, zi12, zi22, S, Lam;
};
#define SHGB_A2_FIELDS(F) F(q) F(p) F(Pq) F(Pp) F(zr11) F(zr12) F(zr22) F(zi11) F(zi12) F(zi22) F(S) F(Lam)

__host__ __device__ inline A2 a2_zero() {
  A2 r;
#define F(f) r.f = 0.0;
  SHGB_A2_FIELDS(F)
#undef F
  return r;
}
__host__ __device__ inline void a2_axpy(A2 &y, double a, const A2 &x) {   // y += a x
#define F(f) y.f += a * x.f;
  SHGB_A2_FIELDS(F)
#undef F
}
__host__ __device__ inline double a2_dot(const A2 &x, const A2 &y) {
  double s = 0.0;
#define F(f) s += x.f * y.f;
  SHGB_A2_FIELDS(F)
#undef F
  return s;
}

// Right-hand side of the beam ODEs (Sec. 2.3, eq:shgb_odes) on component l:
// the formulas of the FP64 stepping kernel.
__host__ __device__ inline A2 a2_rhs(const DevModel &md, int l, const A2 &y, const Q1 &k) {
  const double v = y.p * md.inv_mass;
  const double sg = comp_sigma(l), bc = comp_bcoef(l);
  const double E1 = sg * k.s1, E2 = sg * k.s2, E3 = sg * k.s3;
  const double b0 = bc * k.s, b1 = bc * k.s1, b2 = bc * k.s2;
  A2 d;
  d.q = v;
  d.p = -E1;
  d.Pq = b1 + E2 * y.Pp;
  d.Pp = -y.Pq * md.inv_mass;
  d.zr11 = 2.0 * y.zr12 * E2;
  d.zi11 = 2.0 * y.zi12 * E2 - y.Pp * E3 - b2;
  d.zr12 = y.zr22 * E2 - y.zr11 * md.inv_mass;
  d.zi12 = y.zi22 * E2 - y.zi11 * md.inv_mass;
  d.zr22 = -2.0 * y.zr12 * md.inv_mass;
  d.zi22 = -2.0 * y.zi12 * md.inv_mass;
  d.S = b0;
  d.Lam = 2.0 * fabs(v * k.d21);
  return d;
}

// Stage inputs of one RK4 step (the record the reverse sweep needs).
struct A2Rec {
  A2 Y[4];
};

// One classical RK4 step of size h on component l, folded as the stepping
// kernel folds it; the stage inputs go to rec when it is given.
__host__ __device__ inline void a2_rk4(const DevModel &md, int l, const A2 &y, double h, A2 &out, A2Rec *rec) {
  const double h6 = h * (1.0 / 6.0);
  A2 ys = y, acc;
  for (int st = 0; st < 4; ++st) {
    if (rec) rec->Y[st] = ys;
    const Q1 k = qcle_q1(md, ys.q);
    const A2 d = a2_rhs(md, l, ys, k);
    const double c = st == 2 ? h : 0.5 * h;
    if (st == 0) {
#define F(f) acc.f = d.f; ys.f = y.f + c * d.f;
      SHGB_A2_FIELDS(F)
#undef F
    } else if (st < 3) {
#define F(f) acc.f = acc.f + 2.0 * d.f; ys.f = y.f + c * d.f;
      SHGB_A2_FIELDS(F)
#undef F
    } else {
#define F(f) acc.f = y.f + h6 * (acc.f + d.f);
      SHGB_A2_FIELDS(F)
#undef F
    }
  }
  out = acc;
}

// Vector-Jacobian product of the right-hand side at the stage value y:
// returns g^T d(rhs)/dy and adds g^T d(rhs)/d(A, B, C, D) to th.  The rate
// |v d21| is differentiated with its sign at the value.
__host__ __device__ inline A2 a2_vjp(const DevModel &md, int l, const A2 &y, const A2 &g, double th[4]) {
  const Q1 k = qcle_q1(md, y.q);
  const double im = md.inv_mass, v = y.p * im;
  const double sg = comp_sigma(l), bc = comp_bcoef(l);
  const double E2 = sg * k.s2, E3 = sg * k.s3;
  double sb[5];
  sb[0] = bc * g.S;
  sb[1] = -sg * g.p + bc * g.Pq;
  const double E2b = y.Pp * g.Pq + 2.0 * y.zr12 * g.zr11 + 2.0 * y.zi12 * g.zi11 + y.zr22 * g.zr12 + y.zi22 * g.zi12;
  sb[2] = sg * E2b - bc * g.zi11;
  sb[3] = -sg * y.Pp * g.zi11;
  const double vk = v * k.d21;
  const double sgn = vk > 0.0 ? 1.0 : (vk < 0.0 ? -1.0 : 0.0);
  sb[4] = 2.0 * sgn * v * g.Lam;
  A2 r = a2_zero();
  r.p = (g.q + 2.0 * sgn * k.d21 * g.Lam) * im;
  r.Pq = -g.Pp * im;
  r.Pp = E2 * g.Pq - E3 * g.zi11;
  r.zr11 = -g.zr12 * im;
  r.zi11 = -g.zi12 * im;
  r.zr12 = 2.0 * E2 * g.zr11 - 2.0 * im * g.zr22;
  r.zi12 = 2.0 * E2 * g.zi11 - 2.0 * im * g.zi22;
  r.zr22 = E2 * g.zr12;
  r.zi22 = E2 * g.zi12;
  r.q = q1_pullback_rev(md, y.q, sb, th);
  return r;
}

// Reverse sweep of one RK4 step: given the adjoint yb of its result, the
// adjoint of its start (ybi) and, when need_h, of its step size (hb).
__host__ __device__ inline void a2_rk4_rev(const DevModel &md, int l, const A2Rec &rec, double h, const A2 &yb,
                                           bool need_h, A2 &ybi, double &hb, double th[4]) {
  const double h6 = h * (1.0 / 6.0);
  ybi = yb;
  A2 g = a2_zero();
  a2_axpy(g, h6, yb);
  const A2 Yb4 = a2_vjp(md, l, rec.Y[3], g, th);
  a2_axpy(ybi, 1.0, Yb4);
  g = a2_zero();
  a2_axpy(g, 2.0 * h6, yb);
  a2_axpy(g, h, Yb4);
  const A2 Yb3 = a2_vjp(md, l, rec.Y[2], g, th);
  a2_axpy(ybi, 1.0, Yb3);
  g = a2_zero();
  a2_axpy(g, 2.0 * h6, yb);
  a2_axpy(g, 0.5 * h, Yb3);
  const A2 Yb2 = a2_vjp(md, l, rec.Y[1], g, th);
  a2_axpy(ybi, 1.0, Yb2);
  g = a2_zero();
  a2_axpy(g, h6, yb);
  a2_axpy(g, 0.5 * h, Yb2);
  a2_axpy(ybi, 1.0, a2_vjp(md, l, rec.Y[0], g, th));
  hb = 0.0;
  if (need_h) {
    A2 k[4];
    for (int i = 0; i < 4; ++i) k[i] = a2_rhs(md, l, rec.Y[i], qcle_q1(md, rec.Y[i].q));
    A2 K = k[0];
    a2_axpy(K, 2.0, k[1]);
    a2_axpy(K, 2.0, k[2]);
    a2_axpy(K, 1.0, k[3]);
    hb = a2_dot(yb, K) * (1.0 / 6.0) + a2_dot(Yb4, k[2]) + 0.5 * a2_dot(Yb3, k[1]) + 0.5 * a2_dot(Yb2, k[0]);
  }
}

// Run one interval from (y, h) as the stepping kernel does (Sec. 2.4 steps
// 3-5), completing each hop where it starts.  With stop >= 0 the run stops
// at the start of leg `stop` if the interval gets that far; rem is then the
// time left.  Returns the number of legs run.
__host__ __device__ inline int a2_legs(const DevModel &md, A2 &y, HopScalars &h, uint64_t gid, uint64_t seed,
                                       double dt, int stop, double &rem, Counters &cnt) {
  rem = dt;
  int leg = 0;
  for (;;) {
    if (leg == stop) return leg;
    A2 yt;
    a2_rk4(md, h.comp, y, rem, yt, nullptr);
    if (leg >= SHGB_HOP_CAP || !(yt.Lam >= h.E)) {
      y = yt;
      return leg + 1;
    }
    const double t = (h.E <= y.Lam) ? 0.0 : (h.E - y.Lam) / (yt.Lam - y.Lam);
    if (t > 0.0 && t < 1.0) {
      A2 yp;
      a2_rk4(md, h.comp, y, t * rem, yp, nullptr);
      y = yp;
    } else if (t >= 1.0) {
      y = yt;
    }
    h.logw += y.Lam;
    y.Lam = 0.0;
    const Q1 k = qcle_q1(md, y.q);
    hop_choose(y.p * md.inv_mass * k.d21, h, gid, seed, cnt, kTieRel);
    rem = rem * (1.0 - t);
    ++leg;
    if (!(rem > 0.0)) return leg;
  }
}

// Reverse sweep of one interval that starts at (ys, hs): yb is the adjoint
// of the interval's end state on entry and of its start on return; logwb is
// the adjoint of the final log weight (every hop adds Lam to it).
__host__ __device__ __noinline__ void a2_interval_rev_general(const DevModel &md, const A2 &ys, const HopScalars &hs,
                                                              uint64_t gid, uint64_t seed, double dt, A2 &yb,
                                                              double logwb, double th[4]) {
  A2 y = ys;
  HopScalars h = hs;
  double rem;
  Counters scratch;
  const int L = a2_legs(md, y, h, gid, seed, dt, -1, rem, scratch);
  double remb = 0.0;   // adjoint of the time left at the start of the next leg
  for (int j = L - 1; j >= 0; --j) {
    y = ys;
    h = hs;
    a2_legs(md, y, h, gid, seed, dt, j, rem, scratch);
    const int l = h.comp;
    A2Rec rt;
    A2 yt, ybi;
    a2_rk4(md, l, y, rem, yt, &rt);
    const bool need = j > 0;   // rem depends on the earlier hop times
    double hb = 0.0, rb = 0.0;
    if (j >= SHGB_HOP_CAP || !(yt.Lam >= h.E)) {          // the trial step ends the interval
      a2_rk4_rev(md, l, rt, rem, yb, need, ybi, hb, th);
      rb = hb;
    } else {
      const double t = (h.E <= y.Lam) ? 0.0 : (h.E - y.Lam) / (yt.Lam - y.Lam);
      A2 ym = yb;   // adjoint before the weight update logw += Lam, Lam = 0
      ym.Lam = logwb;
      if (t > 0.0 && t < 1.0) {                          // shortened step to the hop time
        double tb = -rem * remb;
        rb = (1.0 - t) * remb;
        A2Rec rp;
        A2 yp;
        a2_rk4(md, l, y, t * rem, yp, &rp);
        a2_rk4_rev(md, l, rp, t * rem, ym, true, ybi, hb, th);
        tb += rem * hb;
        rb += t * hb;
        // t = (E - Lam)/(Lam' - Lam), Lam' from the trial step, E fixed
        const double den = yt.Lam - y.Lam;
        ybi.Lam += tb * (t - 1.0) / den;
        A2 e = a2_zero();
        e.Lam = -tb * t / den;
        A2 yb2;
        double hb2 = 0.0;
        a2_rk4_rev(md, l, rt, rem, e, need, yb2, hb2, th);
        a2_axpy(ybi, 1.0, yb2);
        rb += hb2;
      } else if (t >= 1.0) {                             // hop at the end of the trial step
        a2_rk4_rev(md, l, rt, rem, ym, need, ybi, hb, th);
        rb = hb;
      } else {                                           // hop at once, no step
        ybi = ym;
        rb = remb;
      }
    }
    yb = ybi;
    remb = rb;
  }
}

// An interval without a hop (its trial step ends it) swept inline, the
// others by the general sweep.
__host__ __device__ inline void a2_interval_rev(const DevModel &md, const A2 &ys, const HopScalars &hs, uint64_t gid,
                                                uint64_t seed, double dt, A2 &yb, double logwb, double th[4]) {
  A2Rec rt;
  A2 yt;
  a2_rk4(md, hs.comp, ys, dt, yt, &rt);
  if (!(yt.Lam >= hs.E)) {
    A2 ybi;
    double hb;
    a2_rk4_rev(md, hs.comp, rt, dt, yb, false, ybi, hb, th);
    yb = ybi;
    return;
  }
  a2_interval_rev_general(md, ys, hs, gid, seed, dt, yb, logwb, th);
}

// Adjoint of one beam's contribution Re(w c) to the objective, c the beam
// integral (the populations' per-beam term, Sec. 2.3 eq:shgb integrated over
// x) with Z = [[z11, z12], [z12, z22]]:
//   c = norm e^(logw + Lam) ph A e^(iS/eps) det(Z)^(-1/2) e^(-P^T Z^-1 P/(2 eps)),
//   dc = c (tr(G dZ) - u^T dP / eps + i dS / eps + dLam + dlogw),
//   G = -Z^-1 / 2 + u u^T / (2 eps), u = Z^-1 P.
// Returns Re(w c); yb gets the adjoint of the state, logwb that of logw.
__host__ __device__ inline double a2_seed(double eps, double norm, const A2 &y, double logw, cd ph, cd A, cd w, A2 &yb,
                                          double &logwb) {
  const double inv_eps = 1.0 / eps;
  const cd z11 = {y.zr11, y.zi11}, z12 = {y.zr12, y.zi12}, z22 = {y.zr22, y.zi22};
  const cd P1 = {y.Pq, 0.0}, P2 = {y.Pp, 0.0};
  // the value, as the populations kernel forms it (LDL^T of Z)
  const cd l21 = cdiv(z12, z11);
  const cd d2 = csub(z22, cmul(l21, z12));
  const cd w2 = csub(P2, cmul(l21, P1));
  const cd quad = cadd(cdiv(cmul(P1, P1), z11), cdiv(cmul(w2, w2), d2));
  const cd sq = cmul(csqrt_principal(z11), csqrt_principal(d2));
  const cd g = cdiv(cexp(cscale(quad, -0.5 * inv_eps)), sq);
  const double mag = exp(logw + y.Lam);
  double sn, cs;
  sincos(y.S * inv_eps, &sn, &cs);
  const cd c = cscale(cmul(cmul(cmul(cscale(ph, mag), A), {cs, sn}), g), norm);
  const cd wc = cmul(w, c);
  // Z^-1 and u
  const cd det = csub(cmul(z11, z22), cmul(z12, z12));
  const cd i11 = cdiv(z22, det), i12 = cdiv({-z12.re, -z12.im}, det), i22 = cdiv(z11, det);
  const cd u1 = cadd(cmul(i11, P1), cmul(i12, P2)), u2 = cadd(cmul(i12, P1), cmul(i22, P2));
  const double h2e = 0.5 * inv_eps;
  const cd K11 = cmul(wc, cadd(cscale(i11, -0.5), cscale(cmul(u1, u1), h2e)));
  const cd K12 = cmul(wc, cadd(cscale(i12, -0.5), cscale(cmul(u1, u2), h2e)));
  const cd K22 = cmul(wc, cadd(cscale(i22, -0.5), cscale(cmul(u2, u2), h2e)));
  yb = a2_zero();
  yb.zr11 = K11.re;
  yb.zi11 = -K11.im;
  yb.zr12 = 2.0 * K12.re;     // the packed variable stands for both (1,2) and (2,1)
  yb.zi12 = -2.0 * K12.im;
  yb.zr22 = K22.re;
  yb.zi22 = -K22.im;
  yb.Pq = -cmul(wc, u1).re * inv_eps;
  yb.Pp = -cmul(wc, u2).re * inv_eps;
  yb.S = -wc.im * inv_eps;
  yb.Lam = wc.re;
  logwb = wc.re;
  return wc.re;
}

}  // namespace shgb
