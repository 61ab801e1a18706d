// Reverse-mode derivative of the populations for the QCLE with a harmonic
// bath (phase space m = 2d > 2): one wavefront per beam, the pair-group
// layout of the stepping kernels with 64 lanes per beam.
//
// The beam ODEs (Sec. 2.3, eq:shgb_odes; the arrowhead Hessian H of the
// bath model is stated in step_wave.hip) are linear in the Hessian Z = M + iN:
//   Z' = L(Z) + i B,   L(Z) = -Z J - J^T Z,   J = [[0, I/M], [-H, 0]],
// B = e0 e0^T (-P_p0 sigma s''' - beta_l''), with J and B depending on the
// centre only.  For adjoints G of symmetric matrices paired with the whole
// matrix (L = sum over all entries G_ab Z_ab), the adjoint of L is
//   L*(G) = -G J^T - J G = S(L(S(G))),
// S the exchange of the position and momentum blocks
// (S [[A, B], [B^T, C]] = [[C, B^T], [B, A]]): the adjoint of the Hessian
// update is the forward update of the exchanged adjoint, so it runs on the
// same pair-group code (grp_deriv) without the B term.  The dependence of
// L on the centre enters only through H_00 = sigma s''(q1):
//   dL/dH00 = 2 sum_a G_a0 Z_a,d   (both real and imaginary parts),
// and B adds -sigma s''' (Im G_00) to the adjoint of P_p0 and to those of
// s'' and s'''.  The coordinates' adjoints and the pullback of the two-level
// quantities to q1 and (A, B, C, D) follow the right-hand side term by term.
//
// Per beam: the adjoint of its final contribution (c from an LDL-type
// elimination of Z, with G = -Z^-1/2 + u u^T/(2 eps), u = Z^-1 P), then the
// segments last to first: each segment is run forward from its checkpoint
// with every interval's start going to the wave's slot store, and the
// intervals are swept in reverse through their legs (adjoint.h): the trial
// step, the shortened step to the hop time and the weight update, with the
// hop time t = (E - Lam)/(Lam' - Lam) carrying the adjoint of the time left.
// The stage inputs of the step being swept sit in LDS.
#include "adjoint.h"
#include "wave.h"

namespace shgb {

constexpr int kAwLanes = 64;   // one beam per wavefront
constexpr int kAwWaves = 4;    // waves per block
constexpr int64_t kAwMaxBlocks = 512;

template <int D>
struct AwT {
  using C = PG<D, kAwLanes>;
  using Y = PgY<D, kAwLanes, double>;
  using Cx = PgCtx<D, kAwLanes, double>;
  using Lds = PgLds<D, double>;
  static constexpr int M = 2 * D;
  static constexpr int NF = C::NG * kGrpN + 2 * C::NXP + 2;   // doubles per lane of a Y
  static constexpr int NSLOT = NF + 3;                        // + E, comp, nhop
  // stage inputs 1..3 of the step being swept, per lane; the seed's
  // elimination reuses the space
  static constexpr int REC = 3 * NF * kAwLanes;
  static constexpr int ELIM = M * (2 * M + 2) * 2;
  static constexpr int SCR = REC > ELIM ? REC : ELIM;
};

template <int D>
struct AwLds {
  typename AwT<D>::Lds x;
  double scr[AwT<D>::SCR];
};

// ---- per-lane state helpers -------------------------------------------------
template <int D>
__device__ inline void aw_zero(typename AwT<D>::Y &y) {
#pragma unroll
  for (int e = 0; e < AwT<D>::C::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] = 0.0;
#pragma unroll
  for (int j = 0; j < AwT<D>::C::NXP; ++j) y.x[j] = y.p[j] = 0.0;
  y.S = y.Lam = 0.0;
}

template <int D>
__device__ inline void aw_axpy(typename AwT<D>::Y &y, double a, const typename AwT<D>::Y &x) {
#pragma unroll
  for (int e = 0; e < AwT<D>::C::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] += a * x.g[e].v[j];
#pragma unroll
  for (int j = 0; j < AwT<D>::C::NXP; ++j) {
    y.x[j] += a * x.x[j];
    y.p[j] += a * x.p[j];
  }
  y.S += a * x.S;
  y.Lam += a * x.Lam;
}

template <int D>
__device__ inline void aw_put(const typename AwT<D>::Y &y, double *dst, int lane) {   // dst[f * 64 + lane]
  int f = 0;
#pragma unroll
  for (int e = 0; e < AwT<D>::C::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) dst[(f++) * kAwLanes + lane] = y.g[e].v[j];
#pragma unroll
  for (int j = 0; j < AwT<D>::C::NXP; ++j) {
    dst[(f++) * kAwLanes + lane] = y.x[j];
    dst[(f++) * kAwLanes + lane] = y.p[j];
  }
  dst[(f++) * kAwLanes + lane] = y.S;
  dst[(f++) * kAwLanes + lane] = y.Lam;
}

template <int D>
__device__ inline void aw_get(typename AwT<D>::Y &y, const double *src, int lane) {
  int f = 0;
#pragma unroll
  for (int e = 0; e < AwT<D>::C::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] = src[(f++) * kAwLanes + lane];
#pragma unroll
  for (int j = 0; j < AwT<D>::C::NXP; ++j) {
    y.x[j] = src[(f++) * kAwLanes + lane];
    y.p[j] = src[(f++) * kAwLanes + lane];
  }
  y.S = src[(f++) * kAwLanes + lane];
  y.Lam = src[(f++) * kAwLanes + lane];
}

__device__ inline double aw_wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Pairing of two adjoint-shaped values over the whole beam: each pair-group
// slot counted as often as its entry appears in the symmetric matrix
// (off-diagonal entries twice), S and Lam once.
template <int D>
__device__ inline double aw_dot(const typename AwT<D>::Cx &cx, const typename AwT<D>::Y &u,
                                const typename AwT<D>::Y &v) {
  using C = typename AwT<D>::C;
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    if (cx.a[e] < 0) continue;
    const double w = cx.a[e] == cx.b[e] ? 1.0 : 2.0;
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) t += u.g[e].v[j] * v.g[e].v[j];
    s += w * t;
  }
#pragma unroll
  for (int j = 0; j < C::NXP; ++j) s += u.x[j] * v.x[j] + u.p[j] * v.p[j];
  return aw_wave_sum(s) + u.S * v.S + u.Lam * v.Lam;
}

// Stage coefficients from the published stage values (as the FP64 stepping kernel forms them).
template <int D>
__device__ inline StageCoef<double> aw_coef(const DevModel &md, int l, const typename AwT<D>::Lds &s) {
  StageCoef<double> c;
  const Q1 k = qcle_q1(md, s.x[0]);
  c.k = Q1T<double>{k.s, k.s1, k.s2, k.s3, k.d21};
  c.im = md.inv_mass;
  c.sg = comp_sigma(l);
  c.bc = comp_bcoef(l);
  c.H00 = c.sg * c.k.s2;
  c.lam = md.lam;
  c.B00 = -s.p[D] * c.sg * c.k.s3 - c.bc * c.k.s2;
  return c;
}

// Right-hand side at published stage values into k (used for the step-size adjoint).
template <int D>
__device__ inline void aw_rhs(const DevModel &md, int l, const typename AwT<D>::Cx &cx, const typename AwT<D>::Y &y,
                              typename AwT<D>::Y &k, typename AwT<D>::Lds &s) {
  using C = typename AwT<D>::C;
  pg_publish(cx, y, s);
  const StageCoef<double> sc = aw_coef<D>(md, l, s);
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const bool live = cx.a[e] >= 0;
    double d[kGrpN];
    grp_deriv<D, double>(live ? cx.a[e] : 0, live ? cx.b[e] : 0, sc, y.g[e].v, s, d);
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) k.g[e].v[j] = live ? d[j] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < C::NXP; ++j) xp_deriv<D, double>(cx.r + kAwLanes * j, sc, s, k.x[j], k.p[j]);
  k.S = sc.bc * sc.k.s;
  k.Lam = 2.0 * fabs(s.x[D] * sc.im * sc.k.d21);
  wave_lds_sync();
}

// One classical RK4 step of size h on component l, folded as the FP64
// stepping kernel folds it; stage inputs 1..3 go to rec (per lane) when given.
template <int D>
__device__ inline void aw_rk4(const DevModel &md, int l, const typename AwT<D>::Cx &cx, const typename AwT<D>::Y &y,
                              double h, typename AwT<D>::Y &out, typename AwT<D>::Lds &s, double *rec) {
  using C = typename AwT<D>::C;
  typename AwT<D>::Y ys = y;
  const double h6 = h * (1.0 / 6.0);
  for (int st = 0; st < 4; ++st) {
    if (rec && st > 0) aw_put<D>(ys, rec + (st - 1) * AwT<D>::NF * kAwLanes, cx.r);
    pg_publish(cx, ys, s);
    const StageCoef<double> sc = aw_coef<D>(md, l, s);
    const double c = st == 2 ? h : 0.5 * h;
    auto fold = [&](double &a, double &yv, double y0v, double d) {
      if (st == 0) a = d;
      else if (st < 3) a = a + 2.0 * d;
      else a = y0v + h6 * (a + d);
      if (st < 3) yv = y0v + c * d;
    };
#pragma unroll
    for (int e = 0; e < C::NG; ++e) {
      const bool live = cx.a[e] >= 0;
      double d[kGrpN];
      grp_deriv<D, double>(live ? cx.a[e] : 0, live ? cx.b[e] : 0, sc, ys.g[e].v, s, d);
#pragma unroll
      for (int j = 0; j < kGrpN; ++j) fold(out.g[e].v[j], ys.g[e].v[j], y.g[e].v[j], live ? d[j] : 0.0);
    }
#pragma unroll
    for (int j = 0; j < C::NXP; ++j) {
      double dx, dp;
      xp_deriv<D, double>(cx.r + kAwLanes * j, sc, s, dx, dp);
      fold(out.x[j], ys.x[j], y.x[j], dx);
      fold(out.p[j], ys.p[j], y.p[j], dp);
    }
    double unused = 0.0;
    fold(out.S, unused, y.S, sc.bc * sc.k.s);
    fold(out.Lam, unused, y.Lam, 2.0 * fabs(s.x[D] * sc.im * sc.k.d21));
    wave_lds_sync();
  }
}

// Vector-Jacobian product of the right-hand side at stage value y: yb gets
// g^T d(rhs)/dy, th (replicated over the lanes) gets g^T d(rhs)/d(A, B, C, D).
template <int D>
__device__ inline void aw_vjp(const DevModel &md, int l, const typename AwT<D>::Cx &cx, const typename AwT<D>::Y &y,
                              const typename AwT<D>::Y &g, typename AwT<D>::Y &yb, double th[4],
                              typename AwT<D>::Lds &s) {
  using C = typename AwT<D>::C;
  const int lane = cx.r;
  const double q0 = __shfl(y.x[0], 0, 64), p0 = __shfl(y.x[0], D, 64), Pp0 = __shfl(y.p[0], D, 64);
  const Q1 k = qcle_q1(md, q0);
  const double im = md.inv_mass, lam = md.lam;
  const double sg = comp_sigma(l), bc = comp_bcoef(l), H00 = sg * k.s2;
  // the Hessian part: the forward update of the exchanged adjoint, exchanged back
  typename AwT<D>::Y gs;
  aw_zero<D>(gs);
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    gs.g[e].v[kRrR] = g.g[e].v[kPpR];
    gs.g[e].v[kRrI] = g.g[e].v[kPpI];
    gs.g[e].v[kAbR] = g.g[e].v[kBaR];
    gs.g[e].v[kAbI] = g.g[e].v[kBaI];
    gs.g[e].v[kBaR] = g.g[e].v[kAbR];
    gs.g[e].v[kBaI] = g.g[e].v[kAbI];
    gs.g[e].v[kPpR] = g.g[e].v[kRrR];
    gs.g[e].v[kPpI] = g.g[e].v[kRrI];
  }
  pg_publish(cx, gs, s);
  StageCoef<double> c0;
  c0.k = Q1T<double>{k.s, k.s1, k.s2, k.s3, k.d21};
  c0.im = im;
  c0.sg = sg;
  c0.bc = bc;
  c0.H00 = H00;
  c0.lam = lam;
  c0.B00 = 0.0;
  double hb = 0.0;
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const bool live = cx.a[e] >= 0;
    double d[kGrpN];
    grp_deriv<D, double>(live ? cx.a[e] : 0, live ? cx.b[e] : 0, c0, gs.g[e].v, s, d);
    yb.g[e].v[kRrR] = live ? d[kPpR] : 0.0;
    yb.g[e].v[kRrI] = live ? d[kPpI] : 0.0;
    yb.g[e].v[kAbR] = live ? d[kBaR] : 0.0;
    yb.g[e].v[kAbI] = live ? d[kBaI] : 0.0;
    yb.g[e].v[kBaR] = live ? d[kAbR] : 0.0;
    yb.g[e].v[kBaI] = live ? d[kAbI] : 0.0;
    yb.g[e].v[kPpR] = live ? d[kRrR] : 0.0;
    yb.g[e].v[kPpI] = live ? d[kRrI] : 0.0;
    // dL/dH00 = 2 sum_a G_a0 Z_a,d: groups (0, k) hold G_k0 (rr) with Z_k,d (Zrp_k0, slot ba)
    // and G_d+k,0 (Zrp_0k, slot ab) with Z_d+k,d (Zpp_k0)
    if (live && cx.a[e] == 0)
      hb += g.g[e].v[kRrR] * y.g[e].v[kBaR] + g.g[e].v[kRrI] * y.g[e].v[kBaI] + g.g[e].v[kAbR] * y.g[e].v[kPpR] +
            g.g[e].v[kAbI] * y.g[e].v[kPpI];
  }
  wave_lds_sync();
  double Hb = 2.0 * aw_wave_sum(hb);
  const double gi00 = __shfl(g.g[0].v[kRrI], 0, 64);   // Im G_00: group (0, 0) is lane 0's first
  // coordinates: lane c owns X_c and P_c (c < 2D)
  const double gx = g.x[0], gp = g.p[0];
  const double gXp0 = __shfl(gx, D, 64), gPr0 = __shfl(gp, 0, 64);
  const double sumX = aw_wave_sum(lane > D && lane < 2 * D ? gx : 0.0);   // sum_{k>0} g of X_{p_k}
  const double sumP = aw_wave_sum(lane > 0 && lane < D ? gp : 0.0);       // sum_{k>0} g of P_{r_k}
  const int partner = lane < D ? lane + D : (lane < 2 * D ? lane - D : lane);
  const double gxo = __shfl(gx, partner, 64), gpo = __shfl(gp, partner, 64);
  const double v = p0 * im, vk = v * k.d21;
  const double sgn = vk > 0.0 ? 1.0 : (vk < 0.0 ? -1.0 : 0.0);
  const double gL = g.Lam;
  double Xb = 0.0, Pb = 0.0;
  if (lane < D) {
    const int i = lane;
    Xb = i == 0 ? -lam * sumX : -lam * gXp0 - md.bath_k[i] * gxo;
    Pb = -gpo * im;
  } else if (lane < 2 * D) {
    const int i = lane - D;
    Xb = gxo * im + (i == 0 ? 2.0 * sgn * k.d21 * gL * im : 0.0);
    Pb = i == 0 ? H00 * gPr0 + lam * sumP - sg * k.s3 * gi00 : lam * gPr0 + md.bath_k[i] * gpo;
  }
  Hb += Pp0 * gPr0;
  double sb[5];
  sb[0] = bc * g.S;
  sb[1] = -sg * gXp0 + bc * gPr0;
  sb[2] = sg * Hb - bc * gi00;
  sb[3] = -sg * Pp0 * gi00;
  sb[4] = 2.0 * sgn * v * gL;
  const double qb = q1_pullback_rev(md, q0, sb, th);
  yb.x[0] = Xb + (lane == 0 ? qb : 0.0);
  yb.p[0] = Pb;
#pragma unroll
  for (int j = 1; j < C::NXP; ++j) yb.x[j] = yb.p[j] = 0.0;
  yb.S = 0.0;
  yb.Lam = 0.0;
}

// Reverse sweep of one RK4 step whose stage inputs 1..3 are in rec and whose
// start is y: ybi = adjoint of the start, hb = adjoint of h (when need_h).
template <int D>
__device__ inline void aw_rk4_rev(const DevModel &md, int l, const typename AwT<D>::Cx &cx,
                                  const typename AwT<D>::Y &y, const double *rec, double h,
                                  const typename AwT<D>::Y &ybo, bool need_h, typename AwT<D>::Y &ybi, double &hb,
                                  double th[4], typename AwT<D>::Lds &s) {
  using Y = typename AwT<D>::Y;
  const int lane = cx.r;
  const double h6 = h * (1.0 / 6.0);
  ybi = ybo;
  Y g, Yb, Ys;
  hb = 0.0;
  // stage 4 (input rec[2]), then 3, 2, 1; kb carries the adjoint of the previous stage's slope
  aw_zero<D>(g);
  aw_axpy<D>(g, h6, ybo);
  aw_get<D>(Ys, rec + 2 * AwT<D>::NF * kAwLanes, lane);
  aw_vjp<D>(md, l, cx, Ys, g, Yb, th, s);
  aw_axpy<D>(ybi, 1.0, Yb);
  double kdot = 0.0;
  if (need_h) {
    Y k3;
    aw_get<D>(Ys, rec + 1 * AwT<D>::NF * kAwLanes, lane);
    aw_rhs<D>(md, l, cx, Ys, k3, s);
    kdot += aw_dot<D>(cx, Yb, k3);
  }
  aw_zero<D>(g);
  aw_axpy<D>(g, 2.0 * h6, ybo);
  aw_axpy<D>(g, h, Yb);
  aw_get<D>(Ys, rec + 1 * AwT<D>::NF * kAwLanes, lane);
  aw_vjp<D>(md, l, cx, Ys, g, Yb, th, s);
  aw_axpy<D>(ybi, 1.0, Yb);
  if (need_h) {
    Y k2;
    aw_get<D>(Ys, rec, lane);
    aw_rhs<D>(md, l, cx, Ys, k2, s);
    kdot += 0.5 * aw_dot<D>(cx, Yb, k2);
  }
  aw_zero<D>(g);
  aw_axpy<D>(g, 2.0 * h6, ybo);
  aw_axpy<D>(g, 0.5 * h, Yb);
  aw_get<D>(Ys, rec, lane);
  aw_vjp<D>(md, l, cx, Ys, g, Yb, th, s);
  aw_axpy<D>(ybi, 1.0, Yb);
  if (need_h) {
    Y k1;
    aw_rhs<D>(md, l, cx, y, k1, s);
    kdot += 0.5 * aw_dot<D>(cx, Yb, k1);
  }
  aw_zero<D>(g);
  aw_axpy<D>(g, h6, ybo);
  aw_axpy<D>(g, 0.5 * h, Yb);
  aw_vjp<D>(md, l, cx, y, g, Yb, th, s);
  aw_axpy<D>(ybi, 1.0, Yb);
  if (need_h) {
    // ybo . (k1 + 2 k2 + 2 k3 + k4) / 6 = ybo . (out - y) / h with out recomputed
    Y K, kk;
    aw_rhs<D>(md, l, cx, y, K, s);
    aw_get<D>(Ys, rec, lane);
    aw_rhs<D>(md, l, cx, Ys, kk, s);
    aw_axpy<D>(K, 2.0, kk);
    aw_get<D>(Ys, rec + 1 * AwT<D>::NF * kAwLanes, lane);
    aw_rhs<D>(md, l, cx, Ys, kk, s);
    aw_axpy<D>(K, 2.0, kk);
    aw_get<D>(Ys, rec + 2 * AwT<D>::NF * kAwLanes, lane);
    aw_rhs<D>(md, l, cx, Ys, kk, s);
    aw_axpy<D>(K, 1.0, kk);
    hb = aw_dot<D>(cx, ybo, K) * (1.0 / 6.0) + kdot;
  }
}

// Beam-level part of a hop at the state y (replicated over the lanes): the
// weight update and the choice from the coupling (p1/M) d21(q1).
template <int D>
__device__ inline void aw_hop(const DevModel &md, typename AwT<D>::Y &y, HopScalars &h, uint64_t gid, uint64_t seed,
                              Counters &cnt) {
  h.logw += y.Lam;
  y.Lam = 0.0;
  const double q1 = __shfl(y.x[0], 0, 64), p1 = __shfl(y.x[0], D, 64);
  const Q1 k = qcle_q1(md, q1);
  hop_choose(p1 * md.inv_mass * k.d21, h, gid, seed, cnt, kTieRel);
}

// One interval from (y, h) as the FP64 stepping kernel runs it, stopping at
// the start of leg `stop` (if reached); returns the number of legs run.
template <int D>
__device__ inline int aw_legs_general(const DevModel &md, const typename AwT<D>::Cx &cx,
                                            typename AwT<D>::Y &y, HopScalars &h, uint64_t gid, uint64_t seed,
                                            double dt, int stop, double &rem, typename AwT<D>::Lds &s) {
  Counters cnt;
  rem = dt;
  int leg = 0;
  for (;;) {
    if (leg == stop) return leg;
    typename AwT<D>::Y yt;
    aw_rk4<D>(md, h.comp, cx, y, rem, yt, s, nullptr);
    if (leg >= SHGB_HOP_CAP || !(yt.Lam >= h.E)) {
      y = yt;
      return leg + 1;
    }
    const double t = (h.E <= y.Lam) ? 0.0 : (h.E - y.Lam) / (yt.Lam - y.Lam);
    if (t > 0.0 && t < 1.0) {
      typename AwT<D>::Y yp;
      aw_rk4<D>(md, h.comp, cx, y, t * rem, yp, s, nullptr);
      y = yp;
    } else if (t >= 1.0) {
      y = yt;
    }
    aw_hop<D>(md, y, h, gid, seed, cnt);
    rem = rem * (1.0 - t);
    ++leg;
    if (!(rem > 0.0)) return leg;
  }
}

// The whole interval: the trial step inline (most intervals have no hop),
// the rest out of line.
template <int D>
__device__ inline void aw_interval(const DevModel &md, const typename AwT<D>::Cx &cx, typename AwT<D>::Y &y,
                                   HopScalars &h, uint64_t gid, uint64_t seed, double dt, typename AwT<D>::Lds &s) {
  typename AwT<D>::Y yt;
  aw_rk4<D>(md, h.comp, cx, y, dt, yt, s, nullptr);
  if (!(yt.Lam >= h.E)) {
    y = yt;
    return;
  }
  double rem;
  aw_legs_general<D>(md, cx, y, h, gid, seed, dt, -1, rem, s);
}

// Reverse sweep of one interval starting at (ys, hs); yb: adjoint of its end
// on entry, of its start on return.
template <int D>
__device__ inline void aw_interval_rev_general(const DevModel &md, const typename AwT<D>::Cx &cx,
                                       const typename AwT<D>::Y &ys, const HopScalars &hs, uint64_t gid,
                                       uint64_t seed, double dt, typename AwT<D>::Y &yb, double logwb, double th[4],
                                       AwLds<D> &lds) {
  using Y = typename AwT<D>::Y;
  Y y = ys;
  HopScalars h = hs;
  double rem;
  const int L = aw_legs_general<D>(md, cx, y, h, gid, seed, dt, -1, rem, lds.x);
  double remb = 0.0;
  for (int j = L - 1; j >= 0; --j) {
    if (j > 0 || L > 1) {
      y = ys;
      h = hs;
      aw_legs_general<D>(md, cx, y, h, gid, seed, dt, j, rem, lds.x);
    } else {
      y = ys;
      h = hs;
      rem = dt;
    }
    const int l = h.comp;
    Y yt, ybi;
    aw_rk4<D>(md, l, cx, y, rem, yt, lds.x, lds.scr);
    const bool need = j > 0;
    double hb = 0.0, rb = 0.0;
    if (j >= SHGB_HOP_CAP || !(yt.Lam >= h.E)) {
      aw_rk4_rev<D>(md, l, cx, y, lds.scr, rem, yb, need, ybi, hb, th, lds.x);
      rb = hb;
    } else {
      const double t = (h.E <= y.Lam) ? 0.0 : (h.E - y.Lam) / (yt.Lam - y.Lam);
      Y ym = yb;
      ym.Lam = logwb;
      if (t > 0.0 && t < 1.0) {
        double tb = -rem * remb;
        rb = (1.0 - t) * remb;
        const double lamt = yt.Lam, lam0 = y.Lam;
        Y yp;
        aw_rk4<D>(md, l, cx, y, t * rem, yp, lds.x, lds.scr);
        aw_rk4_rev<D>(md, l, cx, y, lds.scr, t * rem, ym, true, ybi, hb, th, lds.x);
        tb += rem * hb;
        rb += t * hb;
        const double den = lamt - lam0;
        ybi.Lam += tb * (t - 1.0) / den;
        Y e;
        aw_zero<D>(e);
        e.Lam = -tb * t / den;
        aw_rk4<D>(md, l, cx, y, rem, yt, lds.x, lds.scr);   // the trial step's stage inputs again
        Y yb2;
        double hb2 = 0.0;
        aw_rk4_rev<D>(md, l, cx, y, lds.scr, rem, e, need, yb2, hb2, th, lds.x);
        aw_axpy<D>(ybi, 1.0, yb2);
        rb += hb2;
      } else if (t >= 1.0) {
        aw_rk4_rev<D>(md, l, cx, y, lds.scr, rem, ym, need, ybi, hb, th, lds.x);
        rb = hb;
      } else {
        ybi = ym;
        rb = remb;
      }
    }
    yb = ybi;
    remb = rb;
  }
}

// An interval without a hop (the trial step ends it) swept inline; the
// others by the general sweep.
template <int D>
__device__ inline void aw_interval_rev(const DevModel &md, const typename AwT<D>::Cx &cx,
                                       const typename AwT<D>::Y &ys, const HopScalars &hs, uint64_t gid,
                                       uint64_t seed, double dt, typename AwT<D>::Y &yb, double logwb, double th[4],
                                       AwLds<D> &lds) {
  typename AwT<D>::Y yt;
  aw_rk4<D>(md, hs.comp, cx, ys, dt, yt, lds.x, lds.scr);
  if (!(yt.Lam >= hs.E)) {
    typename AwT<D>::Y ybi;
    double hb;
    aw_rk4_rev<D>(md, hs.comp, cx, ys, lds.scr, dt, yb, false, ybi, hb, th, lds.x);
    yb = ybi;
    return;
  }
  aw_interval_rev_general<D>(md, cx, ys, hs, gid, seed, dt, yb, logwb, th, lds);
}

// Load one beam's state (trajectory rows of f with leading dimension ld,
// scalar rows in sc) into the lane's pair groups and coordinates.
template <int D>
__device__ inline void aw_load(const typename AwT<D>::Cx &cx, const double *f, const double *sc, int64_t ld, int64_t b,
                               typename AwT<D>::Y &y) {
  using C = typename AwT<D>::C;
  constexpr int M = 2 * D;
  const Layout L(M, ld);
  aw_zero<D>(y);
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const int a = cx.a[e], bb = cx.b[e];
    if (a < 0) continue;
    const int trr = Layout::tri(M, a, bb), tab = Layout::tri(M, a, D + bb), tba = Layout::tri(M, bb, D + a),
              tpp = Layout::tri(M, D + a, D + bb);
    const int row[kGrpN] = {L.Zre(trr), L.Zim(trr), L.Zre(tab), L.Zim(tab),
                            L.Zre(tba), L.Zim(tba), L.Zre(tpp), L.Zim(tpp)};
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] = f[row[j] * ld + b];
  }
  const int c = cx.r;
  if (c < M) {
    y.x[0] = f[L.X(c) * ld + b];
    y.p[0] = f[L.P(c) * ld + b];
  }
  y.S = sc[kRowS * ld + b];
  y.Lam = sc[kRowLam * ld + b];
}

// Adjoint of one beam's contribution Re(w c) (the populations' per-beam term):
//   c = (2 pi eps)^(m/2) e^(logw + Lam) ph A e^(iS/eps) det(Z)^(-1/2) e^(-P^T Z^-1 P/(2 eps)),
//   dc = c (sum_ab G_ab dZ_ab - u^T dP/eps + i dS/eps + dLam + dlogw),
// by Gauss-Jordan elimination of [Z | I | P] without pivoting (Re Z positive
// definite: every leading block is invertible, the pivots are those of the
// LDL^T factorisation and det(Z)^(1/2) is the product of their principal
// roots).  Returns Re(w c) (replicated); yb, logwb as in a2_seed.
template <int D>
__device__ inline double aw_seed(const DevModel &md, const typename AwT<D>::Cx &cx, const typename AwT<D>::Y &y,
                                 double logw, cd ph, cd A, cd w, typename AwT<D>::Y &yb, double &logwb,
                                 AwLds<D> &lds) {
  using C = typename AwT<D>::C;
  constexpr int M = 2 * D, W = 2 * M + 1, RW = W + 1;   // row: Z | I | P (padded)
  double *ar = lds.scr, *ai = lds.scr + M * RW;
  const int lane = cx.r;
  // fill Z from the groups, I and P
  for (int t = lane; t < M * RW; t += kAwLanes) { ar[t] = 0.0; ai[t] = 0.0; }
  wave_lds_sync();
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const int a = cx.a[e], b = cx.b[e];
    if (a < 0) continue;
    const double *v = y.g[e].v;
    ar[a * RW + b] = v[kRrR]; ai[a * RW + b] = v[kRrI];
    ar[b * RW + a] = v[kRrR]; ai[b * RW + a] = v[kRrI];
    ar[a * RW + D + b] = v[kAbR]; ai[a * RW + D + b] = v[kAbI];
    ar[(D + b) * RW + a] = v[kAbR]; ai[(D + b) * RW + a] = v[kAbI];
    ar[b * RW + D + a] = v[kBaR]; ai[b * RW + D + a] = v[kBaI];
    ar[(D + a) * RW + b] = v[kBaR]; ai[(D + a) * RW + b] = v[kBaI];
    ar[(D + a) * RW + D + b] = v[kPpR]; ai[(D + a) * RW + D + b] = v[kPpI];
    ar[(D + b) * RW + D + a] = v[kPpR]; ai[(D + b) * RW + D + a] = v[kPpI];
  }
  if (lane < M) {
    ar[lane * RW + M + lane] = 1.0;
    ar[lane * RW + 2 * M] = y.p[0];
  }
  wave_lds_sync();
  cd sq = {1.0, 0.0};
  for (int kk = 0; kk < M; ++kk) {
    const cd piv = {ar[kk * RW + kk], ai[kk * RW + kk]};
    sq = cmul(sq, csqrt_principal(piv));
    const cd rp = cdiv({1.0, 0.0}, piv);
    // every other row minus its multiple of row kk (columns after kk), then row kk scaled
    for (int t = lane; t < M * W; t += kAwLanes) {
      const int i = t / W, j = t % W;
      if (i == kk || j <= kk) continue;
      const cd f = cmul({ar[i * RW + kk], ai[i * RW + kk]}, rp);
      const cd u = cmul(f, {ar[kk * RW + j], ai[kk * RW + j]});
      ar[i * RW + j] -= u.re;
      ai[i * RW + j] -= u.im;
    }
    wave_lds_sync();
    for (int j = lane; j < W; j += kAwLanes) {
      if (j <= kk) continue;
      const cd u = cmul({ar[kk * RW + j], ai[kk * RW + j]}, rp);
      ar[kk * RW + j] = u.re;
      ai[kk * RW + j] = u.im;
    }
    wave_lds_sync();
  }
  // columns M..2M-1: Z^-1; column 2M: u = Z^-1 P
  const double inv_eps = 1.0 / md.eps;
  double quad_r = 0.0, quad_i = 0.0;
  if (lane < M) {
    quad_r = y.p[0] * ar[lane * RW + 2 * M];
    quad_i = y.p[0] * ai[lane * RW + 2 * M];
  }
  const cd quad = {aw_wave_sum(quad_r), aw_wave_sum(quad_i)};
  const cd gq = cdiv(cexp(cscale(quad, -0.5 * inv_eps)), sq);
  const double mag = exp(logw + y.Lam);
  double sn, cs;
  sincos(y.S * inv_eps, &sn, &cs);
  const double norm = pow(2.0 * M_PI * md.eps, 0.5 * M);
  const cd c = cscale(cmul(cmul(cmul(cscale(ph, mag), A), {cs, sn}), gq), norm);
  const cd wc = cmul(w, c);
  const double h2e = 0.5 * inv_eps;
  auto Kat = [&](int i, int j) {   // w c G_ij, G = -Z^-1/2 + u u^T/(2 eps)
    const cd zi = {ar[i * RW + M + j], ai[i * RW + M + j]};
    const cd ui = {ar[i * RW + 2 * M], ai[i * RW + 2 * M]}, uj = {ar[j * RW + 2 * M], ai[j * RW + 2 * M]};
    return cmul(wc, cadd(cscale(zi, -0.5), cscale(cmul(ui, uj), h2e)));
  };
  aw_zero<D>(yb);
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const int a = cx.a[e], b = cx.b[e];
    if (a < 0) continue;
    const cd krr = Kat(a, b), kab = Kat(a, D + b), kba = Kat(b, D + a), kpp = Kat(D + a, D + b);
    yb.g[e].v[kRrR] = krr.re;
    yb.g[e].v[kRrI] = -krr.im;
    yb.g[e].v[kAbR] = kab.re;
    yb.g[e].v[kAbI] = -kab.im;
    yb.g[e].v[kBaR] = kba.re;
    yb.g[e].v[kBaI] = -kba.im;
    yb.g[e].v[kPpR] = kpp.re;
    yb.g[e].v[kPpI] = -kpp.im;
  }
  if (lane < M) {
    const cd ul = {ar[lane * RW + 2 * M], ai[lane * RW + 2 * M]};
    yb.p[0] = -cmul(wc, ul).re * inv_eps;
  }
  yb.S = -wc.im * inv_eps;
  yb.Lam = wc.re;
  logwb = wc.re;
  wave_lds_sync();
  return wc.re;
}

template <int D>
int64_t aw_blocks(int64_t n) {
  int64_t b = (n + kAwWaves - 1) / kAwWaves;
  if (b < 1) b = 1;
  return b < kAwMaxBlocks ? b : kAwMaxBlocks;
}

template <int D>
int64_t aw_workspace_bytes(int64_t n, int every) {
  const int64_t waves = aw_blocks<D>(n) * kAwWaves;
  return waves * (int64_t)every * AwT<D>::NSLOT * kAwLanes * 8 + aw_blocks<D>(n) * kAdjVals * 8;
}

template <int D>
__global__ void __launch_bounds__(kAwLanes * kAwWaves)
adjoint_wave_kernel(DevModel md, const double *__restrict__ fin, const int32_t *__restrict__ fcomp, int64_t n,
                    int64_t ld, uint64_t gid0, const char *__restrict__ ckpt, CkptLayout cl, int nsteps, double dt,
                    uint64_t seed, int every, const double *__restrict__ cot, double inv_ntraj,
                    double *__restrict__ slots, double *__restrict__ partial) {
  using C = typename AwT<D>::C;
  using Y = typename AwT<D>::Y;
  constexpr int M = 2 * D;
  __shared__ AwLds<D> lds_all[kAwWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  AwLds<D> &lds = lds_all[wid];
  const int64_t nwaves = (int64_t)gridDim.x * kAwWaves;
  const int64_t wv = (int64_t)blockIdx.x * kAwWaves + wid;
  double *myslots = slots + wv * (int64_t)every * AwT<D>::NSLOT * kAwLanes;
  typename AwT<D>::Cx cx;
  cx.r = lane;
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const int gi = lane + kAwLanes * e;
    cx.a[e] = cx.b[e] = -1;
    if (gi < C::NGRP) {
      int a = 0, rem = gi;
      while (rem >= D - a) { rem -= D - a; ++a; }
      cx.a[e] = a;
      cx.b[e] = a + rem;
    }
  }
  pg_fill_const<D, kAwLanes, double>(lane, md.bath_k, lds.x);
  const int64_t tro = (int64_t)(2 * M + M * (M + 1));   // trajectory rows
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t b = wv; b < n; b += nwaves) {   // uniform across the wave
    Y y, yb;
    aw_load<D>(cx, fin, fin + tro * ld, ld, b, y);
    const double *fs = fin + tro * ld;
    const int l = fcomp[b];
    const cd w = {cot[2 * l] * inv_ntraj, -cot[2 * l + 1] * inv_ntraj};
    double logwb;
    const double val = aw_seed<D>(md, cx, y, fs[kRowLogw * ld + b], {fs[kRowPhre * ld + b], fs[kRowPhim * ld + b]},
                                  {fs[kRowAre * ld + b], fs[kRowAim * ld + b]}, w, yb, logwb, lds);
    double th[4] = {0.0, 0.0, 0.0, 0.0};
    const uint64_t gid = gid0 + (uint64_t)b;
    for (int c = cl.n_ckpt - 1; c >= 0; --c) {
      const int start = c * every, len = nsteps - start < every ? nsteps - start : every;
      const char *base = ckpt + (int64_t)c * cl.stride_bytes;
      const double *cf = (const double *)base;
      const int32_t *ci = (const int32_t *)(base + cl.rows * n * 8);
      Y ys;
      aw_load<D>(cx, cf, cf + tro * n, n, b, ys);
      HopScalars hs;
      hs.logw = 0.0;
      hs.phre = 1.0;
      hs.phim = 0.0;
      hs.Lam = 0.0;
      hs.E = cf[(tro + kRowE) * n + b];
      hs.comp = ci[b];
      hs.nhop = (uint32_t)ci[n + b];
      for (int i = 0; i < len; ++i) {
        double *sl = myslots + (int64_t)i * AwT<D>::NSLOT * kAwLanes;
        aw_put<D>(ys, sl, lane);
        if (lane == 0) {
          sl[AwT<D>::NF * kAwLanes] = hs.E;
          sl[(AwT<D>::NF + 1) * kAwLanes] = (double)hs.comp;
          sl[(AwT<D>::NF + 2) * kAwLanes] = (double)hs.nhop;
        }
        aw_interval<D>(md, cx, ys, hs, gid, seed, dt, lds.x);
      }
      for (int i = len - 1; i >= 0; --i) {
        const double *sl = myslots + (int64_t)i * AwT<D>::NSLOT * kAwLanes;
        aw_get<D>(ys, sl, lane);
        hs.E = sl[AwT<D>::NF * kAwLanes];
        hs.comp = (int)sl[(AwT<D>::NF + 1) * kAwLanes];
        hs.nhop = (uint32_t)sl[(AwT<D>::NF + 2) * kAwLanes];
        aw_interval_rev<D>(md, cx, ys, hs, gid, seed, dt, yb, logwb, th, lds);
      }
    }
    if (lane == 0) {
      acc[0] += th[0];
      acc[1] += th[1];
      acc[2] += th[2];
      acc[3] += th[3];
      acc[5] += val;
    }
    const double pb = __shfl(yb.x[0], D, 64);   // adjoint of the initial p1
    if (lane == 0) acc[4] += pb;
  }
  __shared__ double red[kAwWaves][6];
  if (lane == 0)
    for (int k = 0; k < 6; ++k) red[wid][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < kAdjVals) {
    double s = 0.0;
    if (threadIdx.x < 6)
      for (int w2 = 0; w2 < kAwWaves; ++w2) s += red[w2][threadIdx.x];
    partial[(int64_t)blockIdx.x * kAdjVals + threadIdx.x] = s;
  }
}

hipError_t launch_adj_final(const double *, int64_t, double *, hipStream_t);

template <int D>
hipError_t launch_aw(const DevModel &md, const shgb_state &fin, const void *ckpt, int nsteps, double dt, uint64_t seed,
                     int every, const double *cot, int64_t n_traj, double *out, void *work, hipStream_t stream) {
  const int64_t n = fin.n_beams;
  const int64_t blocks = aw_blocks<D>(n);
  double *slots = (double *)work;
  double *partial = slots + blocks * kAwWaves * (int64_t)every * AwT<D>::NSLOT * kAwLanes;
  const CkptLayout cl = ckpt_layout(n, 2 * D, nsteps, every);
  hipLaunchKernelGGL(adjoint_wave_kernel<D>, dim3((unsigned)blocks), dim3(kAwLanes * kAwWaves), 0, stream, md,
                     fin.f64, fin.comp, n, fin.ld, fin.beam_id_offset, (const char *)ckpt, cl, nsteps, dt, seed, every,
                     cot, 1.0 / (double)n_traj, slots, partial);
  return launch_adj_final(partial, blocks, out, stream);
}

bool adjoint_wave_supported(int d) { return d == 2 || d == 3 || d == 4 || d == 12; }

int64_t adj_wave_workspace_bytes(int64_t n, int m, int every) {
  switch (m / 2) {
    case 2: return aw_workspace_bytes<2>(n, every);
    case 3: return aw_workspace_bytes<3>(n, every);
    case 4: return aw_workspace_bytes<4>(n, every);
    case 12: return aw_workspace_bytes<12>(n, every);
    default: return -1;
  }
}

hipError_t launch_adjoint_wave(const DevModel &md, const shgb_state &fin, const void *ckpt, int nsteps, double dt,
                               uint64_t seed, int every, const double *cot, int64_t n_traj, double *out, void *work,
                               hipStream_t stream) {
  switch (md.d) {
    case 2: return launch_aw<2>(md, fin, ckpt, nsteps, dt, seed, every, cot, n_traj, out, work, stream);
    case 3: return launch_aw<3>(md, fin, ckpt, nsteps, dt, seed, every, cot, n_traj, out, work, stream);
    case 4: return launch_aw<4>(md, fin, ckpt, nsteps, dt, seed, every, cot, n_traj, out, work, stream);
    case 12: return launch_aw<12>(md, fin, ckpt, nsteps, dt, seed, every, cot, n_traj, out, work, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace shgb
