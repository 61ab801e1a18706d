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
// segments last to first, over chunks of beams: the seed kernel (one
// wavefront per beam); per segment the replay from its checkpoint by the
// FP64 stepping kernel, which writes each interval's stage records (what the
// vector-Jacobian products read of a stage value: q1, p1, the momentum
// component of P and the column d of Z; adjoint.h) and whether the interval
// has a hop; and the reverse kernel (one wavefront per beam), which takes the
// intervals without a hop from their records alone (four stage products per
// RK4 step) and the few with one out of line: their start found again from
// the checkpoint, then swept through their legs (adjoint.h): the trial step,
// the shortened step to the hop time and the weight update, with the hop time
// t = (E - Lam)/(Lam' - Lam) carrying the adjoint of the time left.
#include "adjoint.h"
#include "dual.h"
#include "wave.h"

namespace shgb {

constexpr int kAwLanes = 64;   // one beam per wavefront
constexpr int kAwWaves = 4;    // waves per block

template <int D>
struct AwT {
  using C = PG<D, kAwLanes>;
  using Y = PgY<D, kAwLanes, double>;
  using Cx = PgCtx<D, kAwLanes, double>;
  using Lds = PgLds<D, double>;
  static constexpr int M = 2 * D;
  static constexpr int NF = C::NG * kGrpN + 2 * C::NXP + 2;   // doubles per lane of a Y
  static constexpr int NSLOT = NF + 4;                        // + E, comp, nhop, hop flag
  // What the vector-Jacobian product reads of a stage value: q1, p1 and the
  // momentum component of P (the centre enters through them only), and the
  // column d of Z: Zrp_a0 and Zpp_0a for a < d (the Hessian enters only
  // through dL/dH00).  One record per RK4 stage.
  static constexpr int SR = adj_stage_rec(D);
  static constexpr int RREC = 4 * SR;                         // one RK4 step
  // full stage inputs 1..3 of a step with a hop (the step-size adjoint needs
  // the slopes), per lane, in the wave's workspace
  static constexpr int REC = 3 * NF * kAwLanes;
  // the seed's elimination of [Z | I | P], in LDS
  static constexpr int ELIM = M * (2 * M + 2) * 2;
  // the exchange buffer with the out-of-line hop intervals: the adjoint
  // state and the parameter adjoints
  static constexpr int IO = NF * kAwLanes + 8;
};

// Doubles per beam of the buffers of an interval with a hop: its full stage
// inputs, its stage records and the exchange buffer io.
template <int D>
__host__ __device__ inline int64_t aw_gen_doubles() {
  return AwT<D>::REC + AwT<D>::RREC + AwT<D>::IO;
}

template <int D>
struct AwLds {
  typename AwT<D>::Lds x;
  double scr[AwT<D>::ELIM];
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

// A DPP move of a double within 16-lane rows (CTRL: a DPP control code).
template <int CTRL>
__device__ inline double aw_dpp(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane `src`'s value, read into scalar registers (src uniform).
__device__ inline double aw_lane(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The sum over lanes 0..31 (the lanes that can hold the summed values:
// 2d <= 32), returned to every lane: within each 16-lane row by DPP
// (exchanges with lane ^ 1, lane ^ 2, then rotations by 4 and 8), then the
// two rows' sums read out of lanes 0 and 16.  No LDS traffic.
__device__ inline double aw_sum32(double x) {
  x += aw_dpp<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += aw_dpp<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += aw_dpp<0x124>(x);   // row_ror 4
  x += aw_dpp<0x128>(x);   // row_ror 8
  return aw_lane(x, 0) + aw_lane(x, 16);
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

// The stage record of stage value y (AwT::SR doubles at q): q1, p1, P_p1
// from the lanes that own them, then Zrp_a0 and Zpp_0a of group (0, a) from
// lane a, one row of d values per part.
template <int D>
__device__ inline void aw_record(const typename AwT<D>::Cx &cx, const typename AwT<D>::Y &y, double *q) {
  const int r = cx.r;
  if (r == 0) q[0] = y.x[0];
  if (r == D) {
    q[1] = y.x[0];
    q[2] = y.p[0];
  }
  if (r < D) {
    q[3 + r] = y.g[0].v[kBaR];
    q[3 + D + r] = y.g[0].v[kBaI];
    q[3 + 2 * D + r] = y.g[0].v[kPpR];
    q[3 + 3 * D + r] = y.g[0].v[kPpI];
  }
}

// One classical RK4 step of size h on component l, folded as the FP64
// stepping kernel folds it; stage inputs 1..3 go to rec (per lane) and the
// four stage records to rr, when given.
template <int D>
__device__ inline void aw_rk4(const DevModel &md, int l, const typename AwT<D>::Cx &cx, const typename AwT<D>::Y &y,
                              double h, typename AwT<D>::Y &out, typename AwT<D>::Lds &s, double *rec,
                              double *rr = nullptr) {
  using C = typename AwT<D>::C;
  typename AwT<D>::Y ys = y;
  const double h6 = h * (1.0 / 6.0);
#pragma nounroll
  for (int st = 0; st < 4; ++st) {
    if (rec && st > 0) aw_put<D>(ys, rec + (st - 1) * AwT<D>::NF * kAwLanes, cx.r);
    if (rr) aw_record<D>(cx, ys, rr + st * AwT<D>::SR);
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

// The two-level quantities at the four stages of a step and their Jacobian
// in (q1, A, B, C, D): per stage 32 doubles, (s, s1, s2, s3, d21) then
// J[o][k] at 5 + 5 o + k (o over the five quantities, k over the five
// inputs), in the calling wave's part of an LDS array.
constexpr int kQ1Tab = 32;

template <int D>
__device__ inline double *aw_q1tab() {
  __shared__ double tab[kAwWaves][4 * kQ1Tab];
  return tab[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
}

// Fill the table for the step whose stage records are rr: lane L < 20 takes
// stage L / 5 and the forward derivative along input L % 5 (dual numbers,
// the formulas of the stepping kernels); the values come with every lane.
template <int D>
__device__ inline void aw_q1_fill(const DevModel &md, int lane, const double *rr, double *tab) {
  const int st = lane < 20 ? lane / 5 : 0, k = lane < 20 ? lane % 5 : 0;
  const double q0 = rr[st * AwT<D>::SR];
  QcleDu p;
  p.A = Du(md.A, k == 1 ? 1.0 : 0.0);
  p.B = Du(md.B, k == 2 ? 1.0 : 0.0);
  p.C = Du(md.C, k == 3 ? 1.0 : 0.0);
  p.D = Du(md.D, k == 4 ? 1.0 : 0.0);
  p.inv_mass = md.inv_mass;
  const Q1Du o = qcle_q1_du(p, Du(q0, k == 0 ? 1.0 : 0.0));
  double *t = tab + st * kQ1Tab;
  if (lane < 20) {
    t[5 + k] = o.s.d;
    t[10 + k] = o.s1.d;
    t[15 + k] = o.s2.d;
    t[20 + k] = o.s3.d;
    t[25 + k] = o.d21.d;
    if (k == 0) {
      t[0] = o.s.v;
      t[1] = o.s1.v;
      t[2] = o.s2.v;
      t[3] = o.s3.v;
      t[4] = o.d21.v;
    }
  }
  wave_lds_sync();
}

// The exchange sums of an adjoint that the vector-Jacobian product reads:
// the row sums over k > 0 of Zrp (rho) and of Zpp (chi: the exchanged Zpp is
// written to both triangles, so its row sums are its column sums, term by
// term), one row of 16-byte entries per lane (lanes past the last task
// repeat it), each over four partial sums so that the dependent adds after
// the reads are shorter.  The coordinate sums are not read.
template <int D>
__device__ inline void aw_sums(const typename AwT<D>::Cx &cx, typename AwT<D>::Lds &s) {
  static_assert(2 * D <= kAwLanes, "one exchange sum per lane");
  const int t = cx.r < 2 * D ? cx.r : 2 * D - 1;
  const Cx2<double> *row = t < D ? &s.rp[t][0] : &s.pp[t - D][0];
  Cx2<double> *out = t < D ? &s.rho[t] : &s.chi[t - D];
  double sr[4] = {0.0, 0.0, 0.0, 0.0}, si[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 1; k < D; ++k) {
    const Cx2<double> v = row[k];
    sr[k & 3] += v.re;
    si[k & 3] += v.im;
  }
  *out = Cx2<double>{(sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3])};
}

// Vector-Jacobian product of the right-hand side at the stage value whose
// record is q and whose two-level table is t: yb gets g^T d(rhs)/dy, th
// (replicated over the lanes) gets g^T d(rhs)/d(A, B, C, D).
template <int D>
__device__ inline void aw_vjp(const DevModel &md, int l, const typename AwT<D>::Cx &cx, const double *q,
                              const double *t, const typename AwT<D>::Y &g, typename AwT<D>::Y &yb, double th[4],
                              typename AwT<D>::Lds &s) {
  using C = typename AwT<D>::C;
  const int lane = cx.r;
  const double p0 = q[1], Pp0 = q[2];
  const Q1 k = {t[0], t[1], t[2], t[3], t[4]};
  const double im = md.inv_mass, lam = md.lam;
  const double sg = comp_sigma(l), bc = comp_bcoef(l), H00 = sg * k.s2;
  // the Hessian part: the forward update of the exchanged adjoint, exchanged
  // back; the exchange is done in the writes to the exchange area and per
  // group below (the coordinates of the exchange area are not read here)
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const int a = cx.a[e], b = cx.b[e];
    if ((e + 1) * kAwLanes <= C::NGRP || a >= 0) {
      const double *v = g.g[e].v;
      s.rp[a][b] = Cx2<double>{v[kBaR], v[kBaI]};
      s.rp[b][a] = Cx2<double>{v[kAbR], v[kAbI]};
      s.pp[a][b] = Cx2<double>{v[kRrR], v[kRrI]};
      s.pp[b][a] = Cx2<double>{v[kRrR], v[kRrI]};
    }
  }
  wave_lds_sync();
  aw_sums<D>(cx, s);
  wave_lds_sync();
  StageCoef<double> c0;
  c0.k = Q1T<double>{k.s, k.s1, k.s2, k.s3, k.d21};
  c0.im = im;
  c0.sg = sg;
  c0.bc = bc;
  c0.H00 = H00;
  c0.lam = lam;
  c0.B00 = 0.0;
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const bool live = (e + 1) * kAwLanes <= C::NGRP || cx.a[e] >= 0;   // slots every lane fills need no test
    const double *v = g.g[e].v;
    const double gs[kGrpN] = {v[kPpR], v[kPpI], v[kBaR], v[kBaI], v[kAbR], v[kAbI], v[kRrR], v[kRrI]};
    double d[kGrpN];
    grp_deriv<D, double>(live ? cx.a[e] : 0, live ? cx.b[e] : 0, c0, gs, s, d);
    yb.g[e].v[kRrR] = live ? d[kPpR] : 0.0;
    yb.g[e].v[kRrI] = live ? d[kPpI] : 0.0;
    yb.g[e].v[kAbR] = live ? d[kBaR] : 0.0;
    yb.g[e].v[kAbI] = live ? d[kBaI] : 0.0;
    yb.g[e].v[kBaR] = live ? d[kAbR] : 0.0;
    yb.g[e].v[kBaI] = live ? d[kAbI] : 0.0;
    yb.g[e].v[kPpR] = live ? d[kRrR] : 0.0;
    yb.g[e].v[kPpI] = live ? d[kRrI] : 0.0;
  }
  // dL/dH00 = 2 sum_a G_a0 Z_a,d: group (0, a) (lane a, first slot) holds
  // G_a0 (rr) with Z_a,d (Zrp_a0, slot ba) and G_d+a,0 (Zrp_0a, slot ab)
  // with Z_d+a,d (Zpp_a0)
  double hb = 0.0;
  if (lane < D)
    hb = g.g[0].v[kRrR] * q[3 + lane] + g.g[0].v[kRrI] * q[3 + D + lane] + g.g[0].v[kAbR] * q[3 + 2 * D + lane] +
         g.g[0].v[kAbI] * q[3 + 3 * D + lane];
  wave_lds_sync();
  static_assert(2 * D <= 32, "the centre's sums cover lanes 0..31");
  double Hb = 2.0 * aw_sum32(hb);
  const double gi00 = aw_lane(g.g[0].v[kRrI], 0);   // Im G_00: group (0, 0) is lane 0's first
  // coordinates: lane c owns X_c and P_c (c < 2D)
  const double gx = g.x[0], gp = g.p[0];
  const double gXp0 = aw_lane(gx, D), gPr0 = aw_lane(gp, 0);
  const double sumX = aw_sum32(lane > D && lane < 2 * D ? gx : 0.0);   // sum_{k>0} g of X_{p_k}
  const double sumP = aw_sum32(lane > 0 && lane < D ? gp : 0.0);       // sum_{k>0} g of P_{r_k}
  const int partner = lane < D ? lane + D : (lane < 2 * D ? lane - D : lane);
  const double gxo = __shfl(gx, partner, 64), gpo = __shfl(gp, partner, 64);
  const double v = p0 * im, vk = v * k.d21;
  const double sgn = vk > 0.0 ? 1.0 : (vk < 0.0 ? -1.0 : 0.0);
  const double gL = g.Lam;
  double Xb = 0.0, Pb = 0.0;
  if (lane < D) {
    const int i = lane;
    Xb = i == 0 ? -lam * sumX : -lam * gXp0 - s.hk[i] * gxo;
    Pb = -gpo * im;
  } else if (lane < 2 * D) {
    const int i = lane - D;
    Xb = gxo * im + (i == 0 ? 2.0 * sgn * k.d21 * gL * im : 0.0);
    Pb = i == 0 ? H00 * gPr0 + lam * sumP - sg * k.s3 * gi00 : lam * gPr0 + s.hk[i] * gpo;
  }
  Hb += Pp0 * gPr0;
  double sb[5];
  sb[0] = bc * g.S;
  sb[1] = -sg * gXp0 + bc * gPr0;
  sb[2] = sg * Hb - bc * gi00;
  sb[3] = -sg * Pp0 * gi00;
  sb[4] = 2.0 * sgn * v * gL;
  // the pullback to q1 and (A, B, C, D) through the stage's Jacobian
  double qb = 0.0;
#pragma unroll
  for (int o = 0; o < 5; ++o) qb += sb[o] * t[5 + 5 * o];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double a = 0.0;
#pragma unroll
    for (int o = 0; o < 5; ++o) a += sb[o] * t[5 + 5 * o + 1 + j];
    th[j] += a;
  }
  yb.x[0] = Xb + (lane == 0 ? qb : 0.0);
  yb.p[0] = Pb;
#pragma unroll
  for (int j = 1; j < C::NXP; ++j) yb.x[j] = yb.p[j] = 0.0;
  yb.S = 0.0;
  yb.Lam = 0.0;
}

// Reverse sweep of one RK4 step of size h from its four stage records rr
// (no step-size adjoint): yb holds the adjoint of the step's end on entry
// and that of its start on return.  The stages are swept last to first in a
// loop that is not unrolled, so that one stage's work is live at a time:
// stage i gets the cotangent a_i ybo + b_i Yb_(i+1) (Yb_(i+1) the previous
// product), with (a, b) = (h/6, 0), (h/3, h), (h/3, h/2), (h/6, h/2) for
// stages 4, 3, 2, 1.
template <int D>
__device__ inline void aw_rk4_rev_fast(const DevModel &md, int l, const typename AwT<D>::Cx &cx, const double *rr,
                                       double h, typename AwT<D>::Y &yb, double th[4], typename AwT<D>::Lds &s) {
  using C = typename AwT<D>::C;
  using Y = typename AwT<D>::Y;
  const double h6 = h * (1.0 / 6.0);
  double *tab = aw_q1tab<D>();
  aw_q1_fill<D>(md, cx.r, rr, tab);
  const Y ybo = yb;
  Y Yb;
  aw_zero<D>(Yb);
#pragma nounroll
  for (int st = 3; st >= 0; --st) {
    const double ca = (st == 3 || st == 0) ? h6 : 2.0 * h6;
    const double cb = st == 3 ? 0.0 : (st == 2 ? h : 0.5 * h);
    Y g;
#pragma unroll
    for (int e = 0; e < C::NG; ++e)
#pragma unroll
      for (int j = 0; j < kGrpN; ++j) g.g[e].v[j] = ca * ybo.g[e].v[j] + cb * Yb.g[e].v[j];
#pragma unroll
    for (int j = 0; j < C::NXP; ++j) {
      g.x[j] = ca * ybo.x[j] + cb * Yb.x[j];
      g.p[j] = ca * ybo.p[j] + cb * Yb.p[j];
    }
    g.S = ca * ybo.S + cb * Yb.S;
    g.Lam = ca * ybo.Lam + cb * Yb.Lam;
    aw_vjp<D>(md, l, cx, rr + st * AwT<D>::SR, tab + st * kQ1Tab, g, Yb, th, s);
    aw_axpy<D>(yb, 1.0, Yb);
  }
}

// Reverse sweep of one RK4 step whose stage records are in rr, whose stage
// inputs 1..3 are in rec and whose start is y: ybi = adjoint of the start,
// hb = adjoint of h (when need_h).
template <int D>
__device__ inline void aw_rk4_rev(const DevModel &md, int l, const typename AwT<D>::Cx &cx,
                                  const typename AwT<D>::Y &y, const double *rec, const double *rr, double h,
                                  const typename AwT<D>::Y &ybo, bool need_h, typename AwT<D>::Y &ybi, double &hb,
                                  double th[4], typename AwT<D>::Lds &s) {
  using Y = typename AwT<D>::Y;
  const int lane = cx.r;
  const double h6 = h * (1.0 / 6.0);
  double *tab = aw_q1tab<D>();
  aw_q1_fill<D>(md, lane, rr, tab);
  ybi = ybo;
  Y g, Yb, Ys;
  hb = 0.0;
  // stage 4 (input rec[2]), then 3, 2, 1; kb carries the adjoint of the previous stage's slope
  aw_zero<D>(g);
  aw_axpy<D>(g, h6, ybo);
  aw_vjp<D>(md, l, cx, rr + 3 * AwT<D>::SR, tab + 3 * kQ1Tab, g, Yb, th, s);
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
  aw_vjp<D>(md, l, cx, rr + 2 * AwT<D>::SR, tab + 2 * kQ1Tab, g, Yb, th, s);
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
  aw_vjp<D>(md, l, cx, rr + AwT<D>::SR, tab + kQ1Tab, g, Yb, th, s);
  aw_axpy<D>(ybi, 1.0, Yb);
  if (need_h) {
    Y k1;
    aw_rhs<D>(md, l, cx, y, k1, s);
    kdot += 0.5 * aw_dot<D>(cx, Yb, k1);
  }
  aw_zero<D>(g);
  aw_axpy<D>(g, h6, ybo);
  aw_axpy<D>(g, 0.5 * h, Yb);
  aw_vjp<D>(md, l, cx, rr, tab, g, Yb, th, s);
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

// Orders the wave's own global-memory writes before its later reads of the
// same workspace (the exchange with the out-of-line parts, the replay's
// records before the reverse sweep): a workgroup-scope fence waits for the
// stores to complete.
__device__ inline void aw_mem_sync() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }

// The exchange area of the calling wave, as one LDS array shared by the
// replay and reverse kernels and the out-of-line parts they call (which then
// address it as LDS, not through generic pointers).
template <int D>
__device__ inline typename AwT<D>::Lds &aw_lds() {
  __shared__ typename AwT<D>::Lds lds_all[kAwWaves];
  return lds_all[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
}

// The lane's pair groups: lane r owns groups r + 64 e (a <= b in row order).
template <int D>
__device__ inline typename AwT<D>::Cx aw_ctx(int lane) {
  using C = typename AwT<D>::C;
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
  return cx;
}

// Makes the lane's group context opaque to the compiler at the top of an
// interval, so that the exchange-area and workspace addresses derived from
// it are formed again in each interval rather than held (and spilled) over
// the whole kernel.
template <int D>
__device__ inline void aw_opaque(typename AwT<D>::Cx &cx) {
  asm volatile("" : "+v"(cx.r));
#pragma unroll
  for (int e = 0; e < AwT<D>::C::NG; ++e) asm volatile("" : "+v"(cx.a[e]), "+v"(cx.b[e]));
}

// The out-of-line part (an interval with a hop: a few in a thousand)
// exchanges its state with the calling loop through the beam's buffer io:
// the adjoint state at io and the parameter adjoints at io + NF 64, so that
// the loop's registers are not tied to memory.
// Reverse sweep of one interval starting at (ys, hs); yb: adjoint of its end
// on entry, of its start on return.
template <int D>
__device__ inline void aw_interval_rev_general(const DevModel &md, const typename AwT<D>::Cx &cx,
                                       const typename AwT<D>::Y &ys, const HopScalars &hs, uint64_t gid,
                                       uint64_t seed, double dt, typename AwT<D>::Y &yb, double logwb, double th[4],
                                       typename AwT<D>::Lds &s, double *rec, double *rr) {
  using Y = typename AwT<D>::Y;
  Y y = ys;
  HopScalars h = hs;
  double rem;
  const int L = aw_legs_general<D>(md, cx, y, h, gid, seed, dt, -1, rem, s);
  double remb = 0.0;
  for (int j = L - 1; j >= 0; --j) {
    if (j > 0 || L > 1) {
      y = ys;
      h = hs;
      aw_legs_general<D>(md, cx, y, h, gid, seed, dt, j, rem, s);
    } else {
      y = ys;
      h = hs;
      rem = dt;
    }
    const int l = h.comp;
    Y yt, ybi;
    aw_rk4<D>(md, l, cx, y, rem, yt, s, rec, rr);
    aw_mem_sync();
    const bool need = j > 0;
    double hb = 0.0, rb = 0.0;
    if (j >= SHGB_HOP_CAP || !(yt.Lam >= h.E)) {
      aw_rk4_rev<D>(md, l, cx, y, rec, rr, rem, yb, need, ybi, hb, th, s);
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
        aw_rk4<D>(md, l, cx, y, t * rem, yp, s, rec, rr);
        aw_mem_sync();
        aw_rk4_rev<D>(md, l, cx, y, rec, rr, t * rem, ym, true, ybi, hb, th, s);
        tb += rem * hb;
        rb += t * hb;
        const double den = lamt - lam0;
        ybi.Lam += tb * (t - 1.0) / den;
        Y e;
        aw_zero<D>(e);
        e.Lam = -tb * t / den;
        aw_rk4<D>(md, l, cx, y, rem, yt, s, rec, rr);   // the trial step's stage inputs again
        aw_mem_sync();
        Y yb2;
        double hb2 = 0.0;
        aw_rk4_rev<D>(md, l, cx, y, rec, rr, rem, e, need, yb2, hb2, th, s);
        aw_axpy<D>(ybi, 1.0, yb2);
        rb += hb2;
      } else if (t >= 1.0) {
        aw_rk4_rev<D>(md, l, cx, y, rec, rr, rem, ym, need, ybi, hb, th, s);
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

// Hop scalars of a beam at a checkpoint.
__device__ inline HopScalars aw_ckpt_h(const double *cf, const int32_t *ci, int64_t tro, int64_t n, int64_t b) {
  HopScalars hs;
  hs.logw = 0.0;
  hs.phre = 1.0;
  hs.phim = 0.0;
  hs.Lam = 0.0;
  hs.E = cf[(tro + kRowE) * n + b];
  hs.comp = ci[b];
  hs.nhop = (uint32_t)ci[n + b];
  return hs;
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

// Reverse sweep of interval i of a segment that has a hop: its start is
// read from its slot sl (written by the recording stepping kernel) or, when
// it has none, found again by running the segment from its checkpoint
// (cf, ci; the beam's column b); the adjoint of its end is at io (replaced
// by that of its start), the parameter adjoints it adds go to io + NF 64;
// rec and rr hold the stage values of one step.
template <int D>
__device__ __attribute__((noinline)) void aw_interval_rev_hop(const DevModel &md, const double *cf, const int32_t *ci,
                                                              int64_t n, int64_t b, int i, const double *sl,
                                                              double *io, uint64_t gid, uint64_t seed, double dt,
                                                              double logwb, double *rec, double *rr) {
  using Y = typename AwT<D>::Y;
  constexpr int NF = AwT<D>::NF;
  constexpr int M = 2 * D;
  const typename AwT<D>::Cx cx = aw_ctx<D>(threadIdx.x & 63);
  typename AwT<D>::Lds &s = aw_lds<D>();
  const int64_t tro = (int64_t)(2 * M + M * (M + 1));
  Y ys, yb;
  HopScalars hs;
  if (sl) {
    // the slot's trajectory rows as a state of one beam (ld = 1); its S and
    // Lam follow them (aw_load's scalar reads land inside the rows and are
    // replaced)
    aw_load<D>(cx, sl, sl, 1, 0, ys);
    ys.S = sl[tro];
    ys.Lam = sl[tro + 1];
    hs.logw = 0.0;
    hs.phre = 1.0;
    hs.phim = 0.0;
    hs.Lam = 0.0;
    hs.E = sl[tro + 2];
    hs.comp = (int32_t)sl[tro + 3];
    hs.nhop = (uint32_t)sl[tro + 4];
  } else {
    aw_load<D>(cx, cf, cf + tro * n, n, b, ys);
    hs = aw_ckpt_h(cf, ci, tro, n, b);
    for (int k = 0; k < i; ++k) {
      Y yt;
      aw_rk4<D>(md, hs.comp, cx, ys, dt, yt, s, nullptr);
      if (!(yt.Lam >= hs.E)) {
        ys = yt;
      } else {
        double rem;
        aw_legs_general<D>(md, cx, ys, hs, gid, seed, dt, -1, rem, s);
      }
    }
  }
  aw_get<D>(yb, io, cx.r);
  double th[4] = {0.0, 0.0, 0.0, 0.0};
  aw_interval_rev_general<D>(md, cx, ys, hs, gid, seed, dt, yb, logwb, th, s, rec, rr);
  aw_put<D>(yb, io, cx.r);
  if (cx.r == 0)
    for (int k = 0; k < 4; ++k) io[NF * kAwLanes + k] = th[k];
  aw_mem_sync();
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

// ---- kernels -----------------------------------------------------------------
// One wavefront per beam, kAwWaves per block, over a chunk of beams
// [b0, b0 + nb); per beam of the chunk (index w): its row of kAdjVals
// doubles in bsc (the parameter adjoints dA, dB, dC, dD, that of p_mean,
// the objective, the adjoint of logw), its adjoint state in ybuf, the stage
// records of the current segment in recs and the buffers of an interval with
// a hop in gen.
constexpr int kBscLogwb = 6;

template <int D>
__global__ void __launch_bounds__(kAwLanes * kAwWaves)
aw_seed_kernel(DevModel md, const double *__restrict__ fin, const int32_t *__restrict__ fcomp, int64_t ld,
               int64_t b0, int64_t nb, const double *__restrict__ cot, double inv_ntraj, double *__restrict__ ybuf,
               double *__restrict__ bsc) {
  constexpr int M = 2 * D;
  __shared__ AwLds<D> lds_all[kAwWaves];
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t w = (int64_t)blockIdx.x * kAwWaves + wid;
  if (w >= nb) return;   // uniform over the wave
  AwLds<D> &lds = lds_all[wid];
  const typename AwT<D>::Cx cx = aw_ctx<D>(lane);
  pg_fill_const<D, kAwLanes, double>(lane, md.bath_k, lds.x);
  const int64_t b = b0 + w;
  const int64_t tro = (int64_t)(2 * M + M * (M + 1));
  typename AwT<D>::Y y, yb;
  aw_load<D>(cx, fin, fin + tro * ld, ld, b, y);
  const double *fs = fin + tro * ld;
  const int l = fcomp[b];
  const cd wgt = {cot[2 * l] * inv_ntraj, -cot[2 * l + 1] * inv_ntraj};
  double logwb;
  const double val = aw_seed<D>(md, cx, y, fs[kRowLogw * ld + b], {fs[kRowPhre * ld + b], fs[kRowPhim * ld + b]},
                                {fs[kRowAre * ld + b], fs[kRowAim * ld + b]}, wgt, yb, logwb, lds);
  aw_put<D>(yb, ybuf + w * AwT<D>::NF * kAwLanes, lane);
  if (lane < kAdjVals) {
    double v = 0.0;
    if (lane == 5) v = val;
    if (lane == kBscLogwb) v = logwb;
    bsc[b * kAdjVals + lane] = v;
  }
}

// The checkpoint of the chunk's beams [b0, b0 + nb) (rows of n) into a
// state of rows of ld = chunk, for the replay.
__global__ void __launch_bounds__(256) aw_ckpt_load_kernel(const double *__restrict__ cf, const int32_t *__restrict__ ci,
                                                           int64_t n, int64_t rows, int64_t b0, int64_t nb, int64_t ld,
                                                           double *__restrict__ f64, int32_t *__restrict__ comp,
                                                           uint32_t *__restrict__ nhop) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nb) return;
  for (int64_t f = 0; f < rows; ++f) f64[f * ld + w] = cf[f * n + b0 + w];
  comp[w] = ci[b0 + w];
  nhop[w] = (uint32_t)ci[n + b0 + w];
}

// Reverse sweep of the segment from its records; the adjoint state in ybuf
// and the beam's row of bsc are read and written back.  After the first
// segment (start 0) the adjoint of the initial p1 goes to the row.
// Two wavefronts per SIMD: the register file is halved (a few values of the
// interval loop go to scratch, mostly around the out-of-line call) and the
// latencies of the exchange area and of the FP64 chains are hidden by the
// second wavefront (1.29 s against 1.56 s for the d = 12 gradient workload;
// at three wavefronts the spills cost more than the occupancy gains).
// The records of one interval, copied into a per-wave LDS buffer by 16-byte
// buffer loads with an LDS destination (lane l writes bytes [16 l, 16 l + 16)
// of the wave's destination; gfx950), one interval ahead of their use, so
// that the stage products read them from LDS and the copy's latency is spent
// under the previous interval's work.  Two instructions cover the 2048
// bytes of a buffer; reads past the records' end return zeros (the
// descriptor's byte count), so nothing is read out of bounds.
constexpr int kAwRecBuf = 256;   // doubles per buffer
constexpr int kAwBufferFlags = 0x00020000;   // word 3 of a raw (untyped) buffer resource on gfx9

template <int D>
__device__ inline double *aw_recbuf(int k) {
  static_assert(adj_interval_rec(D) <= kAwRecBuf, "one interval's records fit a buffer");
  __shared__ double buf[kAwWaves][2][kAwRecBuf];
  return buf[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)][k];
}

__device__ inline void aw_rec_fetch(const double *src, int64_t avail, double *dst, int lane) {
  typedef __attribute__((address_space(3))) void *lds_ptr;
  const int64_t bytes = avail * 8;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void *)src, 0, (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff), kAwBufferFlags);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)dst, 16, 16 * lane, 0, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(dst + 128), 16, 16 * lane + 1024, 0, 0, 0);
}

template <int D>
__global__ void __launch_bounds__(kAwLanes * kAwWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
aw_reverse_kernel(DevModel md, const char *__restrict__ ckpt, int64_t ckpt_stride, int64_t rows, int64_t n,
                  int nsteps, int every, int c_hi, int c_lo, int64_t b0, int64_t nb, uint64_t gid0, uint64_t seed,
                  double dt, const double *__restrict__ recs, int64_t seg_stride, const double *__restrict__ slots,
                  int64_t slot_stride, double *__restrict__ ybuf, double *__restrict__ bsc,
                  double *__restrict__ gen) {
  using Y = typename AwT<D>::Y;
  constexpr int NF = AwT<D>::NF, RS = adj_interval_rec(D);
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t w = (int64_t)blockIdx.x * kAwWaves + wid;
  if (w >= nb) return;
  typename AwT<D>::Lds &s = aw_lds<D>();
  typename AwT<D>::Cx cx = aw_ctx<D>(lane);
  pg_fill_const<D, kAwLanes, double>(lane, md.bath_k, s);
  const int64_t b = b0 + w;
  const uint64_t gid = gid0 + (uint64_t)b;
  double *g = gen + w * aw_gen_doubles<D>();
  double *io = g + AwT<D>::REC + AwT<D>::RREC;
  double *row = bsc + b * kAdjVals;
  Y yb;
  aw_get<D>(yb, ybuf + w * NF * kAwLanes, lane);
  double th[4] = {row[0], row[1], row[2], row[3]};
  const double logwb = row[kBscLogwb];
  // segments c_hi down to c_lo: checkpoint c at ckpt + c ckpt_stride, its
  // records (every RS doubles per beam) at recs + (c - c_lo) seg_stride, its
  // hop-interval start states (kAdjSlots per beam) at
  // slots + (c - c_lo) slot_stride
  for (int c = c_hi; c >= c_lo; --c) {
    const char *base = ckpt + (int64_t)c * ckpt_stride;
    const double *cf = (const double *)base;
    const int32_t *ci = (const int32_t *)(base + rows * n * 8);
    const int len = nsteps - c * every < every ? nsteps - c * every : every;
    const double *rw = recs + (int64_t)(c - c_lo) * seg_stride + w * (int64_t)every * RS;
    // (the wave's records are rw[0, len RS): interval j's copy may read (len - j) RS doubles)
    if (len > 0) aw_rec_fetch(rw + (int64_t)(len - 1) * RS, RS, aw_recbuf<D>((len - 1) & 1), lane);
    for (int i = len - 1; i >= 0; --i) {
      aw_opaque<D>(cx);
      __builtin_amdgcn_s_waitcnt(0);   // interval i's records have landed (and every earlier access is done)
      if (i > 0)
        aw_rec_fetch(rw + (int64_t)(i - 1) * RS, (int64_t)(len - i + 1) * RS, aw_recbuf<D>((i - 1) & 1), lane);
      const double *r = aw_recbuf<D>(i & 1);
      if (__builtin_expect(r[AwT<D>::RREC + 1] == 0.0, 1)) {   // (the hop path is the cold one)
        aw_rk4_rev_fast<D>(md, (int)r[AwT<D>::RREC], cx, r, dt, yb, th, s);
      } else {
        const double flag = r[AwT<D>::RREC + 1];   // k + 1: the start is in slot k; -1: no slot
        const double *sl = flag > 0.0 ? slots + (int64_t)(c - c_lo) * slot_stride +
                                             (w * kAdjSlots + (int)flag - 1) * (int64_t)adj_slot_doubles(D)
                                       : nullptr;
        aw_put<D>(yb, io, lane);
        aw_mem_sync();
        aw_interval_rev_hop<D>(md, cf, ci, n, b, i, sl, io, gid, seed, dt, logwb, g, g + AwT<D>::REC);
        aw_get<D>(yb, io, lane);
#pragma unroll
        for (int k = 0; k < 4; ++k) th[k] += io[NF * kAwLanes + k];
      }
    }
  }
  aw_put<D>(yb, ybuf + w * NF * kAwLanes, lane);
  const double pb = __shfl(yb.x[0], D, 64);   // adjoint of p1 at the run's start (after segment 0)
  if (lane == 0) {
    row[0] = th[0];
    row[1] = th[1];
    row[2] = th[2];
    row[3] = th[3];
    if (c_lo == 0) row[4] = pb;
  }
}

// Chunk of beams per pass: bounds the workspace (the records of one segment
// for every beam of the chunk: 1648 bytes per beam and interval at d = 12)
// while giving each launch many wavefronts per SIMD.  Large chunks matter: a
// beam with a hop in a segment runs that interval out of line and is the
// wavefront that finishes last, and with 32 wavefronts per slot instead of 4
// the stragglers of one round are absorbed by the next (the d = 12 gradient
// workload's reverse sweep: 1.29 s with chunks of 8192, 1.05 s with 65536).
constexpr int64_t kAwChunk = 65536;

template <int D>
int64_t aw_chunk(int64_t n) {
  return n < kAwChunk ? (n < 1 ? 1 : n) : kAwChunk;
}

// Workspace (doubles): the records and hop-interval slots of one segment
// for the chunk (none when the forward run kept them), the chunk's adjoint
// states, its buffers
// for intervals with a hop, its replay state (shgb_nfields rows, then comp
// and nhop), and one row of kAdjVals per beam.
template <int D>
int64_t aw_workspace_bytes(int64_t n, int every, bool recorded) {
  const int64_t c = aw_chunk<D>(n);
  const int64_t seg = recorded ? 0 : (int64_t)every * adj_interval_rec(D) + (int64_t)kAdjSlots * adj_slot_doubles(D);
  const int64_t dbl = c * (seg + AwT<D>::NF * kAwLanes + aw_gen_doubles<D>() + shgb_nfields(2 * D) + 1) +
                      (n < 1 ? 1 : n) * kAdjVals;
  return dbl * 8;
}

hipError_t launch_adj_final(const double *, int64_t, double *, hipStream_t);
hipError_t launch_step_wave_record(const DevModel &, const shgb_state &, int, double, uint64_t, double *, int,
                                   double *, uint64_t *, hipStream_t);

// kept: the forward run's records of every segment (segment c, beam b,
// interval i at kept + ((c n + b) every + i) adj_interval_rec(d)), then its
// slots (segment c, beam b at
// kept + n_seg n every adj_interval_rec(d) + (c n + b) kAdjSlots adj_slot_doubles(d)),
// or null for the replay of each segment from its checkpoint.
template <int D>
hipError_t launch_aw(const DevModel &md, const shgb_state &fin, const void *ckpt, const double *kept, int nsteps,
                     double dt, uint64_t seed, int every, const double *cot, int64_t n_traj, double *out, void *work,
                     hipStream_t stream) {
  const int64_t n = fin.n_beams;
  const int64_t chunk = aw_chunk<D>(n);
  const CkptLayout cl = ckpt_layout(n, 2 * D, nsteps, every);
  const int64_t seg = (int64_t)every * adj_interval_rec(D);     // record doubles per beam and segment
  const int64_t sdb = (int64_t)kAdjSlots * adj_slot_doubles(D);  // slot doubles per beam and segment
  double *recs = (double *)work;
  double *wslots = recs + (kept ? 0 : chunk * seg);
  double *ybuf = wslots + (kept ? 0 : chunk * sdb);
  double *gen = ybuf + chunk * AwT<D>::NF * kAwLanes;
  double *rf = gen + chunk * aw_gen_doubles<D>();
  int32_t *rcomp = (int32_t *)(rf + chunk * (int64_t)shgb_nfields(2 * D));
  uint32_t *rnhop = (uint32_t *)(rcomp + chunk);
  double *bsc = rf + chunk * ((int64_t)shgb_nfields(2 * D) + 1);
  const double inv_ntraj = 1.0 / (double)n_traj;
  for (int64_t b0 = 0; b0 < n; b0 += chunk) {
    const int64_t nb = n - b0 < chunk ? n - b0 : chunk;
    const unsigned blocks = (unsigned)((nb + kAwWaves - 1) / kAwWaves);
    hipLaunchKernelGGL(aw_seed_kernel<D>, dim3(blocks), dim3(kAwLanes * kAwWaves), 0, stream, md, fin.f64, fin.comp,
                       fin.ld, b0, nb, cot, inv_ntraj, ybuf, bsc);
    shgb_state rs{};
    rs.f64 = rf;
    rs.comp = rcomp;
    rs.nhop = rnhop;
    rs.n_beams = nb;
    rs.ld = chunk;
    rs.beam_id_offset = fin.beam_id_offset + (uint64_t)b0;
    rs.m = 2 * D;
    rs.precision = SHGB_FP64;
    rs.f32 = nullptr;
    const char *ck = (const char *)ckpt;
    if (kept) {
      // every segment in one launch: each wavefront sweeps its beam's segments
      // last to first from the kept records
      if (cl.n_ckpt > 0)
        hipLaunchKernelGGL(aw_reverse_kernel<D>, dim3(blocks), dim3(kAwLanes * kAwWaves), 0, stream, md, ck,
                           cl.stride_bytes, cl.rows, n, nsteps, every, cl.n_ckpt - 1, 0, b0, nb, fin.beam_id_offset,
                           seed, dt, kept + b0 * seg, n * seg, kept + cl.n_ckpt * n * seg + b0 * sdb, n * sdb, ybuf,
                           bsc, gen);
      continue;
    }
    for (int c = cl.n_ckpt - 1; c >= 0; --c) {
      const int start = c * every, len = nsteps - start < every ? nsteps - start : every;
      const char *base = ck + (int64_t)c * cl.stride_bytes;
      const double *cf = (const double *)base;
      const int32_t *ci = (const int32_t *)(base + cl.rows * n * 8);
      hipLaunchKernelGGL(aw_ckpt_load_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, stream, cf, ci, n,
                         cl.rows, b0, nb, chunk, rf, rcomp, rnhop);
      const hipError_t e = launch_step_wave_record(md, rs, len, dt, seed, recs, every, wslots, nullptr, stream);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(aw_reverse_kernel<D>, dim3(blocks), dim3(kAwLanes * kAwWaves), 0, stream, md, ck,
                         cl.stride_bytes, cl.rows, n, nsteps, every, c, c, b0, nb, fin.beam_id_offset, seed, dt, recs,
                         (int64_t)0, wslots, (int64_t)0, ybuf, bsc, gen);
    }
  }
  return launch_adj_final(bsc, n, out, stream);   // n = 0: zeros
}

bool adjoint_wave_supported(int d) { return d == 2 || d == 3 || d == 4 || d == 12; }

int64_t adj_wave_workspace_bytes(int64_t n, int m, int every, bool recorded) {
  switch (m / 2) {
    case 2: return aw_workspace_bytes<2>(n, every, recorded);
    case 3: return aw_workspace_bytes<3>(n, every, recorded);
    case 4: return aw_workspace_bytes<4>(n, every, recorded);
    case 12: return aw_workspace_bytes<12>(n, every, recorded);
    default: return -1;
  }
}

hipError_t launch_adjoint_wave(const DevModel &md, const shgb_state &fin, const void *ckpt, const double *kept,
                               int nsteps, double dt, uint64_t seed, int every, const double *cot, int64_t n_traj,
                               double *out, void *work, hipStream_t stream) {
  switch (md.d) {
    case 2: return launch_aw<2>(md, fin, ckpt, kept, nsteps, dt, seed, every, cot, n_traj, out, work, stream);
    case 3: return launch_aw<3>(md, fin, ckpt, kept, nsteps, dt, seed, every, cot, n_traj, out, work, stream);
    case 4: return launch_aw<4>(md, fin, ckpt, kept, nsteps, dt, seed, every, cot, n_traj, out, work, stream);
    case 12: return launch_aw<12>(md, fin, ckpt, kept, nsteps, dt, seed, every, cot, n_traj, out, work, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace shgb
