// Beam stepping for the d-dimensional QCLE (phase space m = 2d > 2): a group
// of LPB lanes per beam (64/LPB beams per wavefront), all intervals on chip
// (in registers; for FP64 d = 12 two pair-group slots of the interval's
// starting state in LDS).
//
// Model (Sec. 3.3 with a harmonic bath): E_l(r) = Vb(r) + sigma_l s(q1),
// Vb = sum_{k>=1} (M w_k^2 q_k^2 / 2 + lam q1 q_k), so H = Hess E_l is an
// arrowhead matrix: H_00 = sigma s'', H_0k = H_k0 = lam, H_kk = M w_k^2.
// With J = [[0, I/M], [-H, 0]] the beam ODEs of Sec. 2.3 eq:shgb_odes read, for
// Z = [[Zrr, Zrp], [Zrp^T, Zpp]] = M + iN,
//   Zrr' = Zrp H + (Zrp H)^T + i B,   B = e0 e0^T (-P_p0 sigma s''' - beta'')
//   Zrp' = H Zpp - Zrr / M
//   Zpp' = -(Zrp + Zrp^T) / M
//   X'   = (p/M, -grad E_l),  P' = (grad_r beta + H P_p, -P_r / M),
//   S' = beta_l,  Lam' = 2 |v1 d21(q1)|
// and with the arrowhead H:
//   (Zrp H)_ab = Zrp_ab H_b + lam (b > 0 ? Zrp_a0 : rho_a),   rho_a = sum_{k>0} Zrp_ak
//   (H Zpp)_ab = H_a Zpp_ab + lam (a > 0 ? Zpp_0b : chi_b),   chi_b = sum_{k>0} Zpp_kb.
//
// Work split: for every index pair a <= b the "pair group"
// {Zrr_ab, Zrp_ab, Zrp_ba, Zpp_ab} is owned by one lane, which then has every
// local operand of its four derivatives; only Zrp_a0, Zpp_0b and the sums
// rho, chi come from other lanes, through the beam's slice of LDS.  Lane
// r of the group owns X_c and P_c for c = r, r + LPB, ... below m; the
// scalars (S, Lam, the weight, the threshold and the component) are
// replicated over the group, so the hop logic (Sec. 2.4 steps 3-5) is
// uniform within a group (an FP64 beam's log weight, phase and event counts
// sit in LDS, written alike by its lanes).
//
// Precision: an FP64 state is integrated in FP64 throughout.  For a mixed
// state the stage values and the right-hand side are FP32 (the exchange
// area too), each step's increment is formed in FP32 and added to an FP64
// copy of the state held in registers for the whole call; S and Lam are
// FP64 as in the FP64 path.
#include "adjoint.h"
#include "batch.h"
#include "wave.h"

namespace shgb {

__device__ inline Q1T<double> q1_eval(const DevModel &md, const QcleF &, double q) {
  const Q1 k = qcle_q1(md, q);
  return Q1T<double>{k.s, k.s1, k.s2, k.s3, k.d21};
}

__device__ inline Q1T<float> q1_eval(const DevModel &, const QcleF &mf, float q) {
  const Q1f k = qcle_q1f(mf, q);
  return Q1T<float>{k.s, k.s1, k.s2, k.s3, k.d21};
}

// Per-stage scalars on component l (a hop is completed where it starts, see
// pg_interval, so l is fixed over an RK4 step).
template <int D, typename T>
__device__ inline StageCoef<T> stage_coef(const DevModel &md, const QcleF &mf, int l, const PgLds<D, T> &s) {
  StageCoef<T> c;
  c.k = q1_eval(md, mf, s.x[0]);
  c.im = (T)md.inv_mass;
  c.sg = (T)comp_sigma(l);
  c.bc = (T)comp_bcoef(l);
  c.H00 = c.sg * c.k.s2;
  c.lam = (T)md.lam;
  c.B00 = -s.p[D] * c.sg * c.k.s3 - c.bc * c.k.s2;
  return c;
}

// 32-bit LDS addresses.  A workgroup's exchange areas lie below 64 KiB, so
// two addresses share a word.  Complex entries move as one 16-byte vector.
template <typename X>
using Lds3 = __attribute__((address_space(3))) X;
typedef double Dbl2 __attribute__((ext_vector_type(2)));
template <typename X>
__device__ inline uint32_t lds_addr(const X *p) {
  return (uint32_t)(uintptr_t)(const Lds3<X> *)p;
}
__device__ inline double lds_get_d(uint32_t a) { return *(const Lds3<double> *)(size_t)a; }
__device__ inline Cx2<double> lds_get_c(uint32_t a) {
  const Dbl2 v = *(const Lds3<Dbl2> *)(size_t)a;
  return Cx2<double>{v.x, v.y};
}
__device__ inline void lds_put_c(uint32_t a, double re, double im) {
  Dbl2 v;
  v.x = re;
  v.y = im;
  *(Lds3<Dbl2> *)(size_t)a = v;
}

// The LDS addresses of the operands of a lane's pair-group slots (FP64
// stage loop), formed once per call.  Each stage takes them through an
// empty asm statement, so that the compiler does not hoist what it derives
// from them out of the stage loop (the derived addresses would not fit in
// the registers of two wavefronts per SIMD).
template <int D, int LPB>
struct PgAddr {
  static constexpr int NG = PG<D, LPB>::NG;
  uint32_t wr[NG];  // Zrp_ab | Zrp_ba << 16 (the Zpp entries at a fixed distance)
  uint32_t xt[NG];  // the cross operands of (Zrp H)_ab and (Zrp H)_ba: xo | to << 16
  uint32_t uw[NG];  // the cross operands of (H Zpp)_ab and (H Zpp)_ba: uo | wo << 16
  uint32_t hh[NG];  // hk[a] | hk[b] << 16
  uint32_t sum;     // the lane's sum task: its row's entry 0 | the output << 16
  uint32_t home;    // the lane's first pair of home values (see TileLds)
};

// Values of the interval's starting state kept in LDS instead of registers:
// the first HS pair-group slots of an FP64 d = 12 beam (16 values a lane),
// so that the stage loop of two wavefronts per SIMD fits in the register
// file.  Per wavefront, value v of lane l sits at pair v / 2, lane l:
// home + (v / 2) kHomePair + (v % 2) 8 bytes (16-byte lane stride, no bank
// conflicts).
template <int D, typename TS>
constexpr int home_slots() {
  return (D == 12 && sizeof(TS) == sizeof(double)) ? 2 : 0;
}
constexpr uint32_t kHomePair = 64 * 16;
// values v and v + 1 (v even) as one 16-byte access
__device__ inline Cx2<double> home_get2(uint32_t home, int v) { return lds_get_c(home + (v / 2) * kHomePair); }
__device__ inline void home_put2(uint32_t home, int v, double a, double b) {
  lds_put_c(home + (v / 2) * kHomePair, a, b);
}

// A beam's rarely changed scalars in the FP64 stepping loop (log weight,
// unit phase, event counts), in LDS rather than in registers.
struct HopLds {
  double logw, phre, phim;
  uint32_t cnt[5];   // hops, threshold ties, destination ties, cap, zero rate
  uint32_t nhop0;    // the beam's hop count at the launch's start (the recording kernel's slots)
};

// A workgroup's LDS: the exchange areas (first, so that their addresses fit
// in 16 bits, and at their own stride, which sets how the two beams of a
// wavefront fall on the LDS banks), the home values of its wavefronts and
// the beams' hop scalars.
template <int D, int LPB, typename TS, int WPB>
struct TileLds {
  static constexpr int HS = home_slots<D, TS>();
  PgLds<D, TS> ex[WPB * PG<D, LPB>::G];
  Dbl2 home[WPB][HS > 0 ? HS * kGrpN / 2 : 1][64];
  HopLds hop[WPB * PG<D, LPB>::G];
};

template <int D, int LPB>
__device__ inline PgAddr<D, LPB> pg_addr(const PgCtx<D, LPB, double> &cx, const PgLds<D, double> &s) {
  PgAddr<D, LPB> ad;
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e) {
    const int a = cx.a[e] >= 0 ? cx.a[e] : 0, b = cx.a[e] >= 0 ? cx.b[e] : 0;
    const uint32_t xo = lds_addr(b > 0 ? &s.rp[a][0] : &s.rho[a]), to = lds_addr(a > 0 ? &s.rp[b][0] : &s.rho[b]);
    const uint32_t uo = lds_addr(a > 0 ? &s.pp[0][b] : &s.chi[b]), wo = lds_addr(b > 0 ? &s.pp[0][a] : &s.chi[a]);
    ad.wr[e] = lds_addr(&s.rp[a][b]) | lds_addr(&s.rp[b][a]) << 16;
    ad.xt[e] = xo | to << 16;
    ad.uw[e] = uo | wo << 16;
    ad.hh[e] = lds_addr(&s.hk[a]) | lds_addr(&s.hk[b]) << 16;
  }
  // Sum task t = min(r, 2d): the row sums over k > 0 of Zrp (rho_t), of Zpp
  // (chi_{t-d}: Zpp is symmetric and stored in both triangles, so its row
  // sums are its column sums, term by term) and of the coordinate pairs
  // (sx, sp).  Every task reads a row of complex entries 16 bytes apart.
  const int t = cx.r < 2 * D ? cx.r : 2 * D;
  const Cx2<double> *row = t < D ? &s.rp[t][0] : (t < 2 * D ? &s.pp[t - D][0] : &s.xq[0]);
  const uint32_t out = t < D ? lds_addr(&s.rho[t]) : (t < 2 * D ? lds_addr(&s.chi[t - D]) : lds_addr(&s.sx));
  using S = PgLds<D, double>;
  static_assert(offsetof(S, sp) == offsetof(S, sx) + sizeof(double) && offsetof(S, sx) % 16 == 0,
                "sx and sp as one complex entry");
  ad.sum = lds_addr(row) | out << 16;
  return ad;
}

template <int D, int LPB>
__device__ inline void pg_ctx_opaque(PgCtx<D, LPB, double> &cx) {
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e) {
    asm volatile("" : "+v"(cx.a[e]));
    asm volatile("" : "+v"(cx.b[e]));
  }
  asm volatile("" : "+v"(cx.r));
}

template <int D, int LPB>
__device__ inline void pg_addr_opaque(PgAddr<D, LPB> &ad) {
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e) {
    asm volatile("" : "+v"(ad.wr[e]));
    asm volatile("" : "+v"(ad.xt[e]));
    asm volatile("" : "+v"(ad.uw[e]));
    asm volatile("" : "+v"(ad.hh[e]));
  }
  asm volatile("" : "+v"(ad.sum));
  asm volatile("" : "+v"(ad.home));
}

// Publish the stage values (FP64 stage loop): pg_publish with the slots'
// addresses taken from ad.
template <int D, int LPB>
__device__ inline void pg_publish_ad(const PgCtx<D, LPB, double> &cx, const PgAddr<D, LPB> &ad,
                                     const PgY<D, LPB, double> &y, PgLds<D, double> &s) {
  constexpr uint32_t kPp = (uint32_t)(D * (D + 1) * sizeof(Cx2<double>));   // Zpp after Zrp
  static_assert(sizeof(s.rp) == kPp, "Zpp directly after Zrp");
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e) {
    if ((e + 1) * LPB <= PG<D, LPB>::NGRP || cx.a[e] >= 0) {
      const double *v = y.g[e].v;
      const uint32_t ab = ad.wr[e] & 0xffffu, ba = ad.wr[e] >> 16;
      lds_put_c(ab, v[kAbR], v[kAbI]);
      lds_put_c(ba, v[kBaR], v[kBaI]);   // a == b: the same entry, written twice with one value
      lds_put_c(ab + kPp, v[kPpR], v[kPpI]);
      lds_put_c(ba + kPp, v[kPpR], v[kPpI]);
    }
  }
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) {
    const int c = cx.r + LPB * j;
    if (c < 2 * D) {
      s.x[c] = y.x[j];
      s.p[c] = y.p[j];
      if (c < D) s.xq[c].re = y.x[j];      // X_c (entry 0 is not summed)
      else s.xq[c - D].im = y.p[j];        // P_c, c = d + k
    }
  }
  wave_lds_sync();
  if constexpr (2 * D + 1 <= LPB) {
    // the lane's sum task (lanes past the last task repeat it: the same
    // values to the same place), in the order of pg_sum_task
    const uint32_t row = ad.sum & 0xffffu;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int k = 1; k < D; ++k) {
      const Cx2<double> v = lds_get_c(row + 16 * k);
      sr += v.re;
      si += v.im;
    }
    lds_put_c(ad.sum >> 16, sr, si);
  } else {
    pg_sums(cx, s);   // more tasks than lanes: round robin
  }
  wave_lds_sync();
}

// One Runge-Kutta stage of the FP64 path.  The stage values ys have been
// published to s; the derivative k of each owned value is formed and folded
// at once into the accumulator (zero before stage 0) and the next stage:
//   acc += w k (w = 1, 2, 2, 1),  ys = y0 + c k (c = h/2, h/2, h; 0 in the
//   last stage, whose ys is not used)
// and the step's result is y0 + h/6 acc (pg_finish).  Every slot is
// evaluated: a slot without a pair group computes with the operands of
// group (0, 0) values that nothing reads (they are not published, checked
// or stored).  The folds are
// explicit fused multiply-adds, so that every form of the step rounds alike.
// The pair-group derivatives are those of grp_deriv, with operands read
// from the addresses in ad.
template <int D, int LPB, int HS>
__device__ inline void pg_stage(const DevModel &md, const QcleF &mf, int l, const PgCtx<D, LPB, double> &cx,
                                const PgAddr<D, LPB> &ad, const PgY<D, LPB, double> &y0,
                                PgY<D, LPB, double> &ys, PgY<D, LPB, double> &acc, double w, double c,
                                const PgLds<D, double> &s) {
  using C = PG<D, LPB>;
  const StageCoef<double> sc = stage_coef<D, double>(md, mf, l, s);
  const double lam = sc.lam, im = sc.im;
  // The slots one after another: each slot's LDS reads wait (through an
  // empty asm statement) for the previous slot's last result, the first
  // slot's for the two-level quantities, so that the reads of all slots are
  // not issued ahead together (their operands would not fit in the
  // registers of two wavefronts per SIMD).
  double dep0 = sc.H00, dep1 = sc.B00, dep2 = sc.H00;
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    // index 0 occurs in the first slot only (groups (0, b) come first); a
    // slot without a group reads the operands of group (0, 0)
    const bool can0 = e * LPB < D;
    const bool a0 = can0 && cx.a[e] <= 0, b0 = can0 && cx.b[e] <= 0;
    const double *v = ys.g[e].v;
    uint32_t hh = ad.hh[e], xt = ad.xt[e], uw = ad.uw[e], home = ad.home;
    asm volatile("" : "+v"(hh), "+v"(xt), "+v"(uw), "+v"(home) : "v"(dep0), "v"(dep1), "v"(dep2));
    const double hka = lds_get_d(hh & 0xffffu), hkb = lds_get_d(hh >> 16);   // read unconditionally
    const double Ha = a0 ? sc.H00 : hka, Hb = b0 ? sc.H00 : hkb;
    const Cx2<double> xo = lds_get_c(xt & 0xffffu), to = lds_get_c(xt >> 16);
    const Cx2<double> uo = lds_get_c(uw & 0xffffu), wo = lds_get_c(uw >> 16);
    double d[kGrpN];
    // Zrr_ab' = (Zrp H)_ab + (Zrp H)_ba (+ i B at (0, 0))
    double xr = v[kAbR] * Hb, xi = v[kAbI] * Hb;
    xr += lam * xo.re;
    xi += lam * xo.im;
    double tr = v[kBaR] * Ha, ti = v[kBaI] * Ha;
    tr += lam * to.re;
    ti += lam * to.im;
    d[kRrR] = xr + tr;
    d[kRrI] = (xi + ti) + ((a0 && b0) ? sc.B00 : 0.0);
    // Zrp_ab' = (H Zpp)_ab - Zrr_ab / M,  Zrp_ba' = (H Zpp)_ba - Zrr_ba / M
    double ur = Ha * v[kPpR], ui = Ha * v[kPpI];
    ur += lam * uo.re;
    ui += lam * uo.im;
    double wr = Hb * v[kPpR], wi = Hb * v[kPpI];
    wr += lam * wo.re;
    wi += lam * wo.im;
    d[kAbR] = ur - v[kRrR] * im;
    d[kAbI] = ui - v[kRrI] * im;
    d[kBaR] = wr - v[kRrR] * im;
    d[kBaI] = wi - v[kRrI] * im;
    // Zpp_ab' = -(Zrp_ba + Zrp_ab) / M
    d[kPpR] = -(v[kBaR] + v[kAbR]) * im;
    d[kPpI] = -(v[kBaI] + v[kAbI]) * im;
#pragma unroll
    for (int j = 0; j < kGrpN; j += 2) {
      const Cx2<double> h2 = e < HS ? home_get2(home, e * kGrpN + j) : Cx2<double>{y0.g[e].v[j], y0.g[e].v[j + 1]};
      acc.g[e].v[j] = fma(w, d[j], acc.g[e].v[j]);
      ys.g[e].v[j] = fma(c, d[j], h2.re);
      acc.g[e].v[j + 1] = fma(w, d[j + 1], acc.g[e].v[j + 1]);
      ys.g[e].v[j + 1] = fma(c, d[j + 1], h2.im);
    }
    // the slot's results are complete before the next slot's reads
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) asm volatile("" : "+v"(acc.g[e].v[j]), "+v"(ys.g[e].v[j]));
    dep0 = ys.g[e].v[kRrR];
    dep1 = ys.g[e].v[kAbR];
    dep2 = ys.g[e].v[kBaR];
  }
#pragma unroll
  for (int j = 0; j < C::NXP; ++j) {
    double dx, dp;
    xp_deriv<D, double>(cx.r + LPB * j, sc, s, dx, dp);
    acc.x[j] = fma(w, dx, acc.x[j]);
    ys.x[j] = fma(c, dx, y0.x[j]);
    acc.p[j] = fma(w, dp, acc.p[j]);
    ys.p[j] = fma(c, dp, y0.p[j]);
  }
  const double dS = sc.bc * sc.k.s, dL = 2.0 * fabs(s.x[D] * sc.im * sc.k.d21);
  acc.S = fma(w, dS, acc.S);
  acc.Lam = fma(w, dL, acc.Lam);
}

// The step's result from the accumulated slopes: out = y0 + h6 out (the
// first HS slots of y0 at home).
template <int D, int LPB, int HS>
__device__ inline void pg_finish(const PgY<D, LPB, double> &y0, uint32_t home, double h6,
                                 PgY<D, LPB, double> &out) {
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; j += 2) {
      const Cx2<double> h2 = e < HS ? home_get2(home, e * kGrpN + j) : Cx2<double>{y0.g[e].v[j], y0.g[e].v[j + 1]};
      out.g[e].v[j] = fma(h6, out.g[e].v[j], h2.re);
      out.g[e].v[j + 1] = fma(h6, out.g[e].v[j + 1], h2.im);
    }
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) {
    out.x[j] = fma(h6, out.x[j], y0.x[j]);
    out.p[j] = fma(h6, out.p[j], y0.p[j]);
  }
  out.S = fma(h6, out.S, y0.S);
  out.Lam = fma(h6, out.Lam, y0.Lam);
}

// The stage record of stage values y at q (when q is given): the values
// the reverse sweep's vector-Jacobian products read, in the layout of
// adj_stage_rec (adjoint.h): X_1 from lane 0, X_d+1 and P_d+1 from lane d,
// and from lane a < d the slots ba and pp of its first group, (0, a).
template <int D, int LPB>
__device__ inline void pg_record(const PgCtx<D, LPB, double> &cx, const PgY<D, LPB, double> &y, double *q) {
  static_assert(2 * D <= LPB, "the record's owners are the first 2d lanes, first slots");
  if (!q) return;
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

template <int D, int LPB>
__device__ inline void pg_zero(PgY<D, LPB, double> &y) {
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] = 0.0;
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) y.x[j] = y.p[j] = 0.0;
  y.S = y.Lam = 0.0;
}

// One classical RK4 step of the group's beam on its component, into `out`;
// `s` is clobbered.  The four stages run as a loop: one copy of the stage
// code, whose live set (not that of four interleaved stages) decides the
// registers, so that two wavefronts fit on a SIMD.  REC: the stage records
// go to rec when it is given.
template <int D, int LPB, int HS, bool REC = false>
__device__ inline void pg_rk4(const DevModel &md, const QcleF &mf, const HopCtx &hc, PgCtx<D, LPB, double> &cx,
                              PgAddr<D, LPB> &ad, const PgY<D, LPB, double> &y, double h,
                              PgY<D, LPB, double> &out, PgLds<D, double> &s, double *rec = nullptr) {
  constexpr int SR = adj_stage_rec(D);
  PgY<D, LPB, double> ys = y;
#pragma unroll
  for (int e = 0; e < HS; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; j += 2) {
      const Cx2<double> h2 = home_get2(ad.home, e * kGrpN + j);
      ys.g[e].v[j] = h2.re;
      ys.g[e].v[j + 1] = h2.im;
    }
  const int l = hc.h.comp;
  pg_zero(out);
#pragma unroll 1
  for (int st = 0; st < 4; ++st) {
    if constexpr (REC) pg_record(cx, ys, rec ? rec + st * SR : rec);
    pg_ctx_opaque(cx);
    pg_addr_opaque(ad);
    pg_publish_ad(cx, ad, ys, s);
    // the publish and its sums scheduled apart from the stage's arithmetic
    // (3 % on the d = 12 launch; left to itself the scheduler interleaves
    // them in a slower order)
    __builtin_amdgcn_sched_barrier(0);
    pg_stage<D, LPB, HS>(md, mf, l, cx, ad, y, ys, out, (st == 0 || st == 3) ? 1.0 : 2.0,
                         st == 3 ? 0.0 : (st == 2 ? h : 0.5 * h), s);
    wave_lds_sync();
  }
  pg_finish<D, LPB, HS>(y, ad.home, h * (1.0 / 6.0), out);
}

// Mixed precision: one stage with FP32 stage values and accumulator (zero
// before stage 0): acc += w k (w = 1, 2, 2, 1), ys = y0 + c k in FP32 from
// y0 rounded to FP32 (c = h/2, h/2, h; 0 in the last stage); S and Lam
// accumulate in FP64.  pg_rk4_m turns acc into the step's increment h/6 acc.
template <int D, int LPB>
__device__ inline void pg_stage_m(const DevModel &md, const QcleF &mf, int comp,
                                  const PgCtx<D, LPB, float> &cx, const PgY<D, LPB, double> &y0,
                                  PgY<D, LPB, float> &ys, PgY<D, LPB, float> &acc, float w, float c,
                                  const PgLds<D, float> &s) {
  const StageCoef<float> sc = stage_coef<D, float>(md, mf, comp, s);
  auto fold = [&](float &a, float &yv, double y0v, float d) {
    a = fmaf(w, d, a);
    yv = fmaf(c, d, (float)y0v);
  };
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e) {
    if ((e + 1) * LPB <= PG<D, LPB>::NGRP || cx.a[e] >= 0) {   // slots every lane fills need no test
      float d[kGrpN];
      grp_deriv<D, float>(cx.a[e], cx.b[e], sc, ys.g[e].v, s, d);
#pragma unroll
      for (int j = 0; j < kGrpN; ++j) fold(acc.g[e].v[j], ys.g[e].v[j], y0.g[e].v[j], d[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) {
    float dx, dp;
    xp_deriv<D, float>(cx.r + LPB * j, sc, s, dx, dp);
    fold(acc.x[j], ys.x[j], y0.x[j], dx);
    fold(acc.p[j], ys.p[j], y0.p[j], dp);
  }
  acc.S = fma((double)w, (double)(sc.bc * sc.k.s), acc.S);
  acc.Lam = fma((double)w, (double)(2.0f * fabsf(s.x[D] * sc.im * sc.k.d21)), acc.Lam);
}

// Publish FP32 stage values (mixed path): pg_publish with the exchange sums
// as rows of 8-byte complex entries (Zpp's column sums are its row sums;
// the coordinate sums read the pairs (X_k, P_d+k)), one task per lane.
template <int D, int LPB>
__device__ inline void pg_publish_f(const PgCtx<D, LPB, float> &cx, const PgY<D, LPB, float> &y, PgLds<D, float> &s) {
  pg_write(cx, y, s);
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) {
    const int c = cx.r + LPB * j;
    if (c < D) s.xq[c].re = y.x[j];
    else if (c < 2 * D) s.xq[c - D].im = y.p[j];
  }
  wave_lds_sync();
  if constexpr (2 * D + 1 <= LPB) {
    const int t = cx.r < 2 * D ? cx.r : 2 * D;
    const Cx2<float> *row = t < D ? &s.rp[t][0] : (t < 2 * D ? &s.pp[t - D][0] : &s.xq[0]);
    float sr = 0.0f, si = 0.0f;
#pragma unroll
    for (int k = 1; k < D; ++k) {
      const Cx2<float> v = row[k];
      sr += v.re;
      si += v.im;
    }
    if (t < D) s.rho[t] = Cx2<float>{sr, si};
    else if (t < 2 * D) s.chi[t - D] = Cx2<float>{sr, si};
    else { s.sx = sr; s.sp = si; }
  } else {
    pg_sums(cx, s);
  }
  wave_lds_sync();
}

template <int D, int LPB>
__device__ inline void pg_rk4_m(const DevModel &md, const QcleF &mf, HopCtx &hc, Counters &cnt,
                                const PgCtx<D, LPB, float> &cx, const PgY<D, LPB, double> &y, double h,
                                PgY<D, LPB, float> &inc, PgLds<D, float> &s) {
  PgY<D, LPB, float> ys;
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) {
      ys.g[e].v[j] = (float)y.g[e].v[j];
      inc.g[e].v[j] = 0.0f;
    }
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) {
    ys.x[j] = (float)y.x[j];
    ys.p[j] = (float)y.p[j];
    inc.x[j] = inc.p[j] = 0.0f;
  }
  inc.S = inc.Lam = 0.0;
  // the component once per step: the hop scalars live in scratch memory
  // (their address goes to the out-of-line hop), read there by every stage
  // they cost a scratch load each
  const int comp = hc.h.comp;
#pragma unroll 1
  for (int st = 0; st < 4; ++st) {
    pg_publish_f(cx, ys, s);
    pg_stage_m(md, mf, comp, cx, y, ys, inc, (st == 0 || st == 3) ? 1.0f : 2.0f,
               (float)(st == 3 ? 0.0 : (st == 2 ? h : 0.5 * h)), s);
    wave_lds_sync();
  }
  // the increment h/6 acc
  const double h6d = h * (1.0 / 6.0);
  const float h6 = (float)h6d;
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) inc.g[e].v[j] = h6 * inc.g[e].v[j];
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) {
    inc.x[j] = h6 * inc.x[j];
    inc.p[j] = h6 * inc.p[j];
  }
  inc.S = h6d * inc.S;
  inc.Lam = h6d * inc.Lam;
}

template <int D, int LPB>
__device__ inline void pg_add_inc(PgY<D, LPB, double> &y, const PgY<D, LPB, float> &inc) {
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e)
#pragma unroll
    for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] = y.g[e].v[j] + (double)inc.g[e].v[j];
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) {
    y.x[j] = y.x[j] + (double)inc.x[j];
    y.p[j] = y.p[j] + (double)inc.p[j];
  }
  y.S = y.S + inc.S;
  y.Lam = y.Lam + inc.Lam;
}

// The recording kernel's copy of an interval's start state into a slot
// (adjoint.h: the trajectory rows with ld = 1, then S, Lam, E, comp, nhop):
// every lane of the beam writes the values it owns; the first HS pair-group
// slots come from their LDS home (their registers are not kept).
template <int D, int LPB, int HS>
__device__ inline void pg_save_start(const PgCtx<D, LPB, double> &cx, const PgAddr<D, LPB> &ad,
                                     const PgY<D, LPB, double> &y, const HopScalars &h, double *slot) {
  using C = PG<D, LPB>;
  constexpr int M = 2 * D;
  const Layout L(M, 1);
#pragma unroll
  for (int e = 0; e < C::NG; ++e) {
    const int a = cx.a[e], bb = cx.b[e];
    if (a < 0) continue;
    double v[kGrpN];
#pragma unroll
    for (int j = 0; j < kGrpN; j += 2) {
      if (e < HS) {
        const Cx2<double> h2 = home_get2(ad.home, e * kGrpN + j);
        v[j] = h2.re;
        v[j + 1] = h2.im;
      } else {
        v[j] = y.g[e].v[j];
        v[j + 1] = y.g[e].v[j + 1];
      }
    }
    const int trr = Layout::tri(M, a, bb), tab = Layout::tri(M, a, D + bb), tba = Layout::tri(M, bb, D + a),
              tpp = Layout::tri(M, D + a, D + bb);
    const int row[kGrpN] = {L.Zre(trr), L.Zim(trr), L.Zre(tab), L.Zim(tab),
                            L.Zre(tba), L.Zim(tba), L.Zre(tpp), L.Zim(tpp)};
#pragma unroll
    for (int j = 0; j < kGrpN; ++j)
      if (a != bb || (j != kBaR && j != kBaI)) slot[row[j]] = v[j];
  }
#pragma unroll
  for (int j = 0; j < C::NXP; ++j) {
    const int c = cx.r + LPB * j;
    if (c < M) {
      slot[L.X(c)] = y.x[j];
      slot[L.P(c)] = y.p[j];
    }
  }
  if (cx.r == 0) {
    const int T = L.traj_rows();
    slot[T] = y.S;
    slot[T + 1] = y.Lam;
    slot[T + 2] = h.E;
    slot[T + 3] = (double)h.comp;
    slot[T + 4] = (double)h.nhop;
  }
}

// One interval [t_n, t_n + dt] (Sec. 2.4 steps 3-5) for the group's beam: a
// trial RK4 step; if Lam reaches the threshold, the step to the
// interpolated hop time, the hop (at the state reached), and the rest of
// the interval.  MIXED selects the
// mixed-precision step.
template <int D, int LPB, bool MIXED, int HS, bool REC = false>
__device__ inline void pg_interval(const DevModel &md, const QcleF &mf, PgCtx<D, LPB, double> &cx,
                                   const PgCtx<D, LPB, float> &cxf, PgAddr<D, LPB> &ad, int base, PgY<D, LPB, double> &y, HopCtx &hc,
                                   double dt, Counters &cnt, void *lds, HopLds &hl, double *rec = nullptr,
                                   double *hslot = nullptr) {
  const double tie_rel = MIXED ? kTieRelMixed : kTieRel;
  double rem = dt, hstep = dt, theta = 1.0;
  bool partial = false;
  int hops = 0;
  using YN = typename std::conditional<MIXED, PgY<D, LPB, float>, PgY<D, LPB, double>>::type;
  YN yn;  // FP64: the trial result; mixed: the trial increment
  auto trial = [&](double hh, double *rq) {
    if constexpr (MIXED) pg_rk4_m(md, mf, hc, cnt, cxf, y, hh, yn, *(PgLds<D, float> *)lds);
    else pg_rk4<D, LPB, HS, REC>(md, mf, hc, cx, ad, y, hh, yn, *(PgLds<D, double> *)lds, rq);
  };
  // REC: the first trial step's stage records, then the interval's component
  // and whether it has a hop (the trial step is not its whole result)
  const int comp0 = hc.h.comp;
  auto accept = [&]() {
    if constexpr (MIXED) {
      pg_add_inc(y, yn);
    } else {
      y = yn;
#pragma unroll
      for (int e = 0; e < HS; ++e)
#pragma unroll
        for (int j = 0; j < kGrpN; j += 2) home_put2(ad.home, e * kGrpN + j, yn.g[e].v[j], yn.g[e].v[j + 1]);
    }
  };
  for (;;) {
    trial(hstep, (REC && hops == 0 && !partial) ? rec : nullptr);
    const double E = hc.h.E;
    if (!partial) {
      const bool capped = hops >= SHGB_HOP_CAP;
      const double lam_n = MIXED ? y.Lam + yn.Lam : yn.Lam;
      if (!capped && fabs(lam_n - E) <= tie_rel * E) {
        if constexpr (MIXED) cnt.thr_ties++;
        else hl.cnt[1]++;   // every lane of the beam writes the same count
      }
      if constexpr (REC) {
        if (hops == 0 && rec) {
          // the hop flag: 0 no hop, k + 1 the start state in slot k, -1 no slot
          double flag = 0.0;
          if (!capped && lam_n >= E) {
            const uint32_t k = hc.h.nhop - hl.nhop0;
            flag = -1.0;
            if (hslot && k < (uint32_t)kAdjSlots) {
              pg_save_start<D, LPB, HS>(cx, ad, y, hc.h, hslot + (int64_t)k * adj_slot_doubles(D));
              flag = (double)(k + 1);
            }
          }
          if (cx.r == 0) {
            rec[4 * adj_stage_rec(D)] = (double)comp0;
            rec[4 * adj_stage_rec(D) + 1] = flag;
          }
        }
      }
      if (capped || !(lam_n >= E)) {
        if (capped) {
          if constexpr (MIXED) cnt.cap++;
          else hl.cnt[3]++;
        }
        accept();
        break;
      }
      theta = (E <= y.Lam) ? 0.0 : (E - y.Lam) / (lam_n - y.Lam);
      if (theta > 0.0 && theta < 1.0) {
        partial = true;
        hstep = theta * rem;
        continue;
      }
      if (theta >= 1.0) accept();
    } else {
      accept();
      partial = false;
    }
    // the hop at once, from the coupling (p1/M) d21(q1) at the state reached (in
    // the stage precision).  Mixed: the draw and the choice out of line (inline
    // they spill inside the interval loop).  FP64: inline, with the beam's log
    // weight, phase and counts in LDS (HopLds; every lane of the beam
    // computes and writes the same values), so that nothing is held in
    // registers across the interval loop for the hop and no call saves
    // registers in scratch memory.
    if constexpr (MIXED) {
      hop_start(hc, y.Lam);
      const float q1 = (float)__shfl(y.x[0], base, 64),
                  p1 = (float)__shfl(y.x[D / LPB], base + D % LPB, 64);
      const Q1f k = qcle_q1f(mf, q1);
      hop_choose_call((double)(p1 * mf.inv_mass * k.d21), hc.h, hc.gid, hc.seed, cnt, kTieRelMixed);
    } else {
      HopScalars hh = hc.h;
      hh.logw = hl.logw + y.Lam;   // the weight update of hop_start
      hh.phre = hl.phre;
      hh.phim = hl.phim;
      hop_start(hc, y.Lam);
      const double q1 = __shfl(y.x[0], base, 64), p1 = __shfl(y.x[D / LPB], base + D % LPB, 64);
      const Q1 k = qcle_q1(md, q1);
      Counters c1;
      hop_choose(p1 * md.inv_mass * k.d21, hh, hc.gid, hc.seed, c1, kTieRel);
      hl.logw = hh.logw;
      hl.phre = hh.phre;
      hl.phim = hh.phim;
      hl.cnt[0] += c1.hops;
      hl.cnt[2] += c1.dest_ties;
      hl.cnt[4] += c1.zero_rate;
      hc.h.comp = hh.comp;
      hc.h.nhop = hh.nhop;
      hc.h.E = hh.E;
    }
    hc.pending = false;
    ++hops;
    rem = rem * (1.0 - theta);
    if (!(rem > 0.0)) break;
    hstep = rem;
  }
}

constexpr int kWavesPerBlock = 4;
// Lanes per d = 12 beam: 32, two beams per wavefront, two wavefronts per
// SIMD for both precisions.  The FP64 stage runs as a loop over the four
// stages with the slots in sequence and two slots of the interval's state
// in LDS (TileLds), which keeps it within 256 registers without spills; at
// 16 lanes per beam the three copies of the state alone need 276.  The FP32
// stage keeps its branches (branch-free, it spills at two waves per SIMD).
constexpr int kLanesPerBeamD12 = 32;

// All nsteps intervals of the beams of one tile (WPB waves, 64/LPB beams
// per wave).  TS: element type of the stored trajectory rows (double: FP64
// path, float: mixed path); the register copy of the state is FP64 in both.
// The group's replicated counts are added to cnt by its lane 0 only.
template <int D, int LPB, typename TS, int WPB, bool REC = false>
__device__ inline void wave_tile(const DevModel &md, TS *__restrict__ tr, double *__restrict__ sc,
                                 int32_t *__restrict__ comp, uint32_t *__restrict__ nhop, int64_t n, int64_t ld,
                                 uint64_t gid0, int nsteps, double dt, uint64_t seed, int64_t tile,
                                 TileLds<D, LPB, TS, WPB> &tl, Counters &cnt_out, double *__restrict__ recs = nullptr,
                                 int every = 0, double *__restrict__ slots = nullptr) {
  constexpr int HS = TileLds<D, LPB, TS, WPB>::HS;
  PgLds<D, TS> *lds = tl.ex;
  using C = PG<D, LPB>;
  constexpr int M = C::M;
  constexpr bool MIXED = sizeof(TS) == sizeof(float);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = lane / LPB, r = lane % LPB, base = grp * LPB;
  const int slot = wid * C::G + grp;
  constexpr int NB = WPB * C::G;  // beams of the tile
  // A tile narrower than a 128-byte line of a trajectory row writes its rows
  // through LDS after the last interval, all of the tile's beams of a row at
  // once: written by each beam on its own, the line's pieces leave the L2 at
  // different times and are written to HBM more than once.
  constexpr bool kStageOut = NB * (int)sizeof(TS) < 128;
  constexpr int kTrajRows = 2 * M + M * (M + 1);
  static_assert(!kStageOut || kTrajRows * NB * sizeof(TS) <= sizeof(TileLds<D, LPB, TS, WPB>),
                "the tile's trajectory rows fit in its LDS");
  const int64_t b = tile * NB + slot;
  const Layout L(M, ld);
  Counters cnt;
  PgCtx<D, LPB, double> cx;
  PgY<D, LPB, double> y;
  if (b < n) {  // uniform across the beam's lanes
    const QcleF mf = qcle_f32(md);
    PgCtx<D, LPB, float> cxf;
    cx.r = cxf.r = r;
#pragma unroll
    for (int e = 0; e < C::NG; ++e) {
      const int gi = r + LPB * e;
      cx.a[e] = cx.b[e] = -1;
#pragma unroll
      for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] = 0.0;
      if (gi < C::NGRP) {
        int a = 0, rem = gi;
        while (rem >= D - a) { rem -= D - a; ++a; }
        const int bb = a + rem;
        cx.a[e] = a;
        cx.b[e] = bb;
        const int trr = Layout::tri(M, a, bb), tab = Layout::tri(M, a, D + bb), tba = Layout::tri(M, bb, D + a),
                  tpp = Layout::tri(M, D + a, D + bb);
        const int row[kGrpN] = {L.Zre(trr), L.Zim(trr), L.Zre(tab), L.Zim(tab),
                                L.Zre(tba), L.Zim(tba), L.Zre(tpp), L.Zim(tpp)};
#pragma unroll
        for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] = (double)tr[row[j] * ld + b];
      }
      cxf.a[e] = cx.a[e];
      cxf.b[e] = cx.b[e];
    }
#pragma unroll
    for (int j = 0; j < C::NXP; ++j) {
      const int c = r + LPB * j;
      y.x[j] = c < M ? (double)tr[L.X(c) * ld + b] : 0.0;
      y.p[j] = c < M ? (double)tr[L.P(c) * ld + b] : 0.0;
    }
    y.S = sc[kRowS * ld + b];
    y.Lam = sc[kRowLam * ld + b];
    HopCtx hc;
    HopScalars &h = hc.h;
    h.logw = sc[kRowLogw * ld + b];
    h.phre = sc[kRowPhre * ld + b];
    h.phim = sc[kRowPhim * ld + b];
    h.E = sc[kRowE * ld + b];
    h.comp = comp[b];
    h.nhop = nhop[b];
    h.Lam = y.Lam;
    hc.pending = false;
    hc.gid = gid0 + (uint64_t)b;
    hc.seed = seed;
    pg_fill_const<D, LPB>(r, md.bath_k, lds[slot]);
    HopLds &hl = tl.hop[slot];
    if constexpr (!MIXED) {
      // the beam's rarely changed scalars (every lane writes the same values;
      // only the beam's lanes read them, after the first publish's barrier)
      hl.logw = h.logw;
      hl.phre = h.phre;
      hl.phim = h.phim;
#pragma unroll
      for (int t = 0; t < 5; ++t) hl.cnt[t] = 0u;
      hl.nhop0 = h.nhop;
    }
    PgAddr<D, LPB> ad{};
    if constexpr (!MIXED) {
      ad = pg_addr(cx, lds[slot]);
      ad.home = lds_addr(&tl.home[wid][0][lane]);
#pragma unroll
      for (int e = 0; e < HS; ++e)
#pragma unroll
        for (int j = 0; j < kGrpN; j += 2) home_put2(ad.home, e * kGrpN + j, y.g[e].v[j], y.g[e].v[j + 1]);
    }
    for (int st = 0; st < nsteps; ++st)
      pg_interval<D, LPB, MIXED, HS, REC>(md, mf, cx, cxf, ad, base, y, hc, dt, cnt, (void *)&lds[slot], hl,
                                      REC ? recs + ((int64_t)b * every + st) * adj_interval_rec(D) : nullptr,
                                      REC && slots ? slots + (int64_t)b * kAdjSlots * adj_slot_doubles(D) : nullptr);
    // (every hop is completed where it starts, so none is pending here)
    // the beam index through an empty asm statement: the stores' addresses
    // are formed here, not kept from the loads before the interval loop
    int64_t bw = b;
    asm volatile("" : "+v"(bw));
#pragma unroll
    for (int e = 0; e < HS; ++e)
#pragma unroll
      for (int j = 0; j < kGrpN; j += 2) {
        const Cx2<double> h2 = home_get2(ad.home, e * kGrpN + j);
        y.g[e].v[j] = h2.re;
        y.g[e].v[j + 1] = h2.im;
      }
    // finiteness of the values this lane owns (slots without a pair group
    // or coordinate hold no state)
    if constexpr (!MIXED) {
      h.logw = hl.logw;
      h.phre = hl.phre;
      h.phim = hl.phim;
      cnt.hops = hl.cnt[0];
      cnt.thr_ties = hl.cnt[1];
      cnt.dest_ties = hl.cnt[2];
      cnt.cap = hl.cnt[3];
      cnt.zero_rate = hl.cnt[4];
    }
    double chk = y.S + y.Lam + h.logw;
#pragma unroll
    for (int j = 0; j < C::NXP; ++j)
      if (r + LPB * j < M) chk += y.x[j] + y.p[j];
#pragma unroll
    for (int e = 0; e < C::NG; ++e)
      if (cx.a[e] >= 0)
#pragma unroll
        for (int j = 0; j < kGrpN; ++j) chk += y.g[e].v[j];
    int bad = !isfinite(chk);
#pragma unroll
    for (int off = 1; off < LPB; off <<= 1) bad |= __shfl_xor(bad, off, 64);
    if constexpr (!kStageOut) {
#pragma unroll
      for (int e = 0; e < C::NG; ++e) {
        const int a = cx.a[e], bb = cx.b[e];
        if (a >= 0) {
          const int trr = Layout::tri(M, a, bb), tab = Layout::tri(M, a, D + bb), tba = Layout::tri(M, bb, D + a),
                    tpp = Layout::tri(M, D + a, D + bb);
          const int row[kGrpN] = {L.Zre(trr), L.Zim(trr), L.Zre(tab), L.Zim(tab),
                                  L.Zre(tba), L.Zim(tba), L.Zre(tpp), L.Zim(tpp)};
#pragma unroll
          for (int j = 0; j < kGrpN; ++j)
            if (a != bb || (j != kBaR && j != kBaI)) tr[row[j] * ld + bw] = (TS)y.g[e].v[j];
        }
      }
#pragma unroll
      for (int j = 0; j < C::NXP; ++j) {
        const int c = r + LPB * j;
        if (c < M) {
          tr[L.X(c) * ld + bw] = (TS)y.x[j];
          tr[L.P(c) * ld + bw] = (TS)y.p[j];
        }
      }
    }
    if (r == 0) {
      sc[kRowS * ld + bw] = y.S;
      sc[kRowLam * ld + bw] = y.Lam;
      sc[kRowLogw * ld + bw] = h.logw;
      sc[kRowPhre * ld + bw] = h.phre;
      sc[kRowPhim * ld + bw] = h.phim;
      sc[kRowE * ld + bw] = h.E;
      comp[bw] = h.comp;
      nhop[bw] = h.nhop;
      if (bad) cnt.nonfinite++;
      cnt_out.hops += cnt.hops;
      cnt_out.thr_ties += cnt.thr_ties;
      cnt_out.dest_ties += cnt.dest_ties;
      cnt_out.cap += cnt.cap;
      cnt_out.zero_rate += cnt.zero_rate;
      cnt_out.nonfinite += cnt.nonfinite;
    }
  }
  if constexpr (kStageOut) {
    // rows [kTrajRows][NB] over the whole tile area, once every wave of the
    // tile is past its last interval
    TS *stg = reinterpret_cast<TS *>(&tl);
    __syncthreads();
    if (b < n) {
#pragma unroll
      for (int e = 0; e < C::NG; ++e) {
        const int a = cx.a[e], bb = cx.b[e];
        if (a >= 0) {
          const int trr = Layout::tri(M, a, bb), tab = Layout::tri(M, a, D + bb), tba = Layout::tri(M, bb, D + a),
                    tpp = Layout::tri(M, D + a, D + bb);
          const int row[kGrpN] = {L.Zre(trr), L.Zim(trr), L.Zre(tab), L.Zim(tab),
                                  L.Zre(tba), L.Zim(tba), L.Zre(tpp), L.Zim(tpp)};
#pragma unroll
          for (int j = 0; j < kGrpN; ++j)
            if (a != bb || (j != kBaR && j != kBaI)) stg[row[j] * NB + slot] = (TS)y.g[e].v[j];
        }
      }
#pragma unroll
      for (int j = 0; j < C::NXP; ++j) {
        const int c = r + LPB * j;
        if (c < M) {
          stg[L.X(c) * NB + slot] = (TS)y.x[j];
          stg[L.P(c) * NB + slot] = (TS)y.p[j];
        }
      }
    }
    __syncthreads();
    const int64_t b0 = tile * NB;
    for (int i = threadIdx.x; i < kTrajRows * NB; i += 64 * WPB) {
      const int row = i / NB, s = i % NB;
      if (b0 + s < n) tr[row * ld + b0 + s] = stg[i];
    }
  }
}

// The tile of workgroup b when K consecutive tiles share the 128-byte lines
// of the state rows (d = 12: a tile of 8 beams covers half a line of FP64
// rows, a quarter of FP32 rows): consecutive workgroups are dispatched to the
// 8 XCDs in turn, so tiles Ki .. Ki + K-1 go to workgroups b, b + 8, ...,
// which run on one XCD and share its L2, and each line is fetched once.
// Groups of 8K workgroups are permuted; a last partial group keeps its order.
template <int K>
__device__ inline int64_t xcd_line_tile(int64_t b, int64_t nblocks) {
  if constexpr (K <= 1) {
    return b;
  } else {
    const int64_t q = b / (8 * K), r = b % (8 * K);
    if ((q + 1) * (8 * K) > nblocks) return b;
    return 8 * K * q + K * (r % 8) + r / 8;
  }
}

template <int D, int LPB, typename TS>
constexpr int tiles_per_line() {
  constexpr int bytes = kWavesPerBlock * PG<D, LPB>::G * (int)sizeof(TS);
  return bytes >= 128 ? 1 : 128 / bytes;
}

template <int D, int LPB, typename TS>
__global__ void __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(2)))
step_wave_kernel(DevModel md, TS *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
                 uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, int nsteps, double dt,
                 uint64_t seed, uint64_t *diag) {
  __shared__ TileLds<D, LPB, TS, kWavesPerBlock> tl;
  static_assert(sizeof(tl.ex) <= 65536, "16-bit LDS addresses (PgAddr)");
  Counters cnt;
  wave_tile<D, LPB, TS, kWavesPerBlock>(md, tr, sc, comp, nhop, n, ld, gid0, nsteps, dt, seed,
                                        xcd_line_tile<tiles_per_line<D, LPB, TS>()>(blockIdx.x, gridDim.x), tl, cnt);
  flush_counters(cnt, diag);
}

// Persistent form for a batch: each workgroup takes tiles from the queue
// until none is left; the tile decides the instance (model and state).
template <int D, int LPB, typename TS, int WPB>
__global__ void __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(2)))
step_wave_batched(const BatchItem *__restrict__ items, int n_items, int64_t total_tiles, int grab, int nsteps,
                  double dt, unsigned long long *queue, uint64_t *diag) {
  __shared__ TileLds<D, LPB, TS, WPB> tl;
  static_assert(sizeof(tl.ex) <= 65536, "16-bit LDS addresses (PgAddr)");
  Counters cnt;
  for (;;) {
    const int64_t t0 = batch_grab(queue, grab);
    if (t0 >= total_tiles) break;
    const int64_t t1 = t0 + grab < total_tiles ? t0 + grab : total_tiles;
    for (int64_t t = t0; t < t1; ++t) {
      const BatchItem &it = items[batch_find(items, n_items, t)];
      wave_tile<D, LPB, TS, WPB>(it.md, (TS *)it.tr, it.sc, it.comp, it.nhop, it.n, it.ld, it.gid0, nsteps, dt,
                                 it.seed, t - it.tile0, tl, cnt);
      __syncthreads();
    }
  }
  flush_counters(cnt, diag);
}

// The FP64 stepping kernel that also writes, for every interval, the stage
// records of its trial step, its component and its hop flag (the forward run
// that keeps its records, or the replay of a segment for the reverse sweep;
// records of beam b, interval i at recs + (b every + i) adj_interval_rec(d)),
// and the start states of the intervals with a hop in the beam's slots at
// slots + b kAdjSlots adj_slot_doubles(d) (adjoint.h; slots may be null: then
// the flags say "no slot").  One launch is one segment.  diag may be null.
template <int D, int LPB>
__global__ void __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(2)))
step_wave_rec_kernel(DevModel md, double *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
                     uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, int nsteps, double dt,
                     uint64_t seed, double *__restrict__ recs, int every, double *__restrict__ slots,
                     uint64_t *diag) {
  __shared__ TileLds<D, LPB, double, kWavesPerBlock> tl;
  static_assert(sizeof(tl.ex) <= 65536, "16-bit LDS addresses (PgAddr)");
  Counters cnt;
  wave_tile<D, LPB, double, kWavesPerBlock, true>(md, tr, sc, comp, nhop, n, ld, gid0, nsteps, dt, seed,
                                                  xcd_line_tile<tiles_per_line<D, LPB, double>()>(blockIdx.x, gridDim.x),
                                                  tl, cnt, recs, every, slots);
  flush_counters(cnt, diag);
}

template <int D, int LPB>
static void launch_pg_rec(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                          double *recs, int every, double *slots, uint64_t *diag, hipStream_t stream) {
  constexpr int beams_per_block = kWavesPerBlock * PG<D, LPB>::G;
  const int64_t blocks = (st.n_beams + beams_per_block - 1) / beams_per_block;
  hipLaunchKernelGGL((step_wave_rec_kernel<D, LPB>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, stream,
                     md, st.f64, scalar_block(st), st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps,
                     dt, seed, recs, every, slots, diag);
}

hipError_t launch_step_wave_record(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                                   double *recs, int every, double *slots, uint64_t *diag, hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  if (mixed(st) || nsteps > every) return hipErrorInvalidValue;
  switch (md.d) {
    case 2: launch_pg_rec<2, 8>(md, st, nsteps, dt, seed, recs, every, slots, diag, stream); break;
    case 3: launch_pg_rec<3, 8>(md, st, nsteps, dt, seed, recs, every, slots, diag, stream); break;
    case 4: launch_pg_rec<4, 8>(md, st, nsteps, dt, seed, recs, every, slots, diag, stream); break;
    case 12:
      launch_pg_rec<12, kLanesPerBeamD12>(md, st, nsteps, dt, seed, recs, every, slots, diag, stream);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool step_wave_supported(int d) { return d == 2 || d == 3 || d == 4 || d == 12; }

template <int D, int LPB, typename TS>
static void launch_pg_t(const DevModel &md, const shgb_state &st, TS *tr, int nsteps, double dt, uint64_t seed,
                        uint64_t *diag, hipStream_t stream) {
  constexpr int beams_per_block = kWavesPerBlock * PG<D, LPB>::G;
  const int64_t blocks = (st.n_beams + beams_per_block - 1) / beams_per_block;
  hipLaunchKernelGGL((step_wave_kernel<D, LPB, TS>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, stream,
                     md, tr, scalar_block(st), st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt,
                     seed, diag);
}

template <int D, int LPB32, int LPB64>
static void launch_pg(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed, uint64_t *diag,
                      hipStream_t stream) {
  if (mixed(st)) launch_pg_t<D, LPB32, float>(md, st, st.f32, nsteps, dt, seed, diag, stream);
  else launch_pg_t<D, LPB64, double>(md, st, st.f64, nsteps, dt, seed, diag, stream);
}

// beams per tile of the batched wave kernels
int wave_tile_beams(int d, int wpb) { return wpb * 64 / (d == 12 ? kLanesPerBeamD12 : 8); }

template <int D, int LPB, int WPB>
static void launch_pg_batched(bool mixed_state, const BatchItem *items, int n_items, int64_t total_tiles, int grab,
                              int blocks, int nsteps, double dt, unsigned long long *queue, uint64_t *diag,
                              hipStream_t stream) {
  if (mixed_state)
    hipLaunchKernelGGL((step_wave_batched<D, LPB, float, WPB>), dim3(blocks), dim3(64 * WPB), 0, stream, items,
                       n_items, total_tiles, grab, nsteps, dt, queue, diag);
  else
    hipLaunchKernelGGL((step_wave_batched<D, LPB, double, WPB>), dim3(blocks), dim3(64 * WPB), 0, stream, items,
                       n_items, total_tiles, grab, nsteps, dt, queue, diag);
}

hipError_t launch_step_wave_batched(int d, bool mixed_state, int wpb, const BatchItem *items, int n_items,
                                    int64_t total_tiles, int grab, int blocks, int nsteps, double dt,
                                    unsigned long long *queue, uint64_t *diag, hipStream_t stream) {
#define SHGB_PGB(DD, LL)                                                                                     \
  case DD:                                                                                                  \
    if (wpb == 2) launch_pg_batched<DD, LL, 2>(mixed_state, items, n_items, total_tiles, grab, blocks, nsteps, dt, \
                                              queue, diag, stream);                                         \
    else launch_pg_batched<DD, LL, 4>(mixed_state, items, n_items, total_tiles, grab, blocks, nsteps, dt, queue, \
                                      diag, stream);                                                        \
    break;
  switch (d) {
    SHGB_PGB(2, 8)
    SHGB_PGB(3, 8)
    SHGB_PGB(4, 8)
    SHGB_PGB(12, kLanesPerBeamD12)
    default: return hipErrorInvalidValue;
  }
#undef SHGB_PGB
  return hipGetLastError();
}

hipError_t launch_step_wave(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                            uint64_t *diag, hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  switch (md.d) {
    case 2: launch_pg<2, 8, 8>(md, st, nsteps, dt, seed, diag, stream); break;
    case 3: launch_pg<3, 8, 8>(md, st, nsteps, dt, seed, diag, stream); break;
    case 4: launch_pg<4, 8, 8>(md, st, nsteps, dt, seed, diag, stream); break;
    case 12: launch_pg<12, kLanesPerBeamD12, kLanesPerBeamD12>(md, st, nsteps, dt, seed, diag, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace shgb
