// Beam stepping for the one-dimensional QCLE (phase space m = 2): one thread
// per beam, the whole beam state in registers for all nsteps intervals.
//
// Beam ODEs (Sec. 2.3, eq:shgb_odes) on component l, x = (q, p), v = p/M:
//   X' = alpha_l = (v, -E_l'),  J = d alpha_l / dx = [[0, 1/M], [-E_l'', 0]]
//   P' = grad beta_l - J^T P      = (beta_l' + E_l'' P_p, -P_q / M)
//   Z' = -Z J - J^T Z + i (Hess(P.alpha_l) - Hess beta_l),  Z = M + iN,
//        Hess(P.alpha_l) = [[-P_p E_l''', 0], [0, 0]]
//   S' = beta_l,  A' = gamma_ll A = 0,  Lam' = sum_{j != l} |gamma_jl| = 2 |v d21|
// The interval algorithm (Sec. 2.4 steps 3-5) runs one RK4 call site in a
// loop: a trial over the rest of the interval, then, if Lam crosses the
// threshold, the shortened step to the interpolated hop time, the hop, and a
// new trial on the new component.  The hop needs the coupling at the hop
// state, which is exactly where the next RK4 step starts: its stage 0
// evaluates the two-level quantities there anyway (they do not depend on
// the component), so the hop is completed inside that stage.  The weight
// update (logw += Lam, Lam = 0) is done at once; a hop still pending when
// the call ends is completed before the state is stored.
#include "batch.h"

namespace shgb {

struct Ode2 {
  double q, p, Pq, Pp, zr11, zr12, zr22, zi11, zi12, zi22, S, Lam;
};

// One Runge-Kutta stage: the derivative at the stage values ys is folded at
// once into the accumulator and the next stage values,
//   stage 0: acc = k;   stages 1, 2: acc += 2 k;   (ys = y0 + c k)
//   stage 3: acc = y0 + h6 (acc + k)   (the step's result).
// Stage 0 first completes a pending hop at ys = y0.
__host__ __device__ inline void stage2(const DevModel &md, HopCtx &hc, Counters &cnt, const Ode2 &y0, Ode2 &ys,
                                       Ode2 &acc, int stage, double c, double h6) {
  const Q1 k = qcle_q1(md, ys.q);
  const double v = ys.p * md.inv_mass;
  if (stage == 0 && hc.pending) {
    hop_choose(v * k.d21, hc.h, hc.gid, hc.seed, cnt, kTieRel);
    hc.pending = false;
  }
  const int l = hc.h.comp;
  const double sg = comp_sigma(l), bc = comp_bcoef(l);
  const double E1 = sg * k.s1, E2 = sg * k.s2, E3 = sg * k.s3;
  const double b0 = bc * k.s, b1 = bc * k.s1, b2 = bc * k.s2;
  Ode2 d;
  d.q = v;
  d.p = -E1;
  d.Pq = b1 + E2 * ys.Pp;
  d.Pp = -ys.Pq * md.inv_mass;
  d.zr11 = 2.0 * ys.zr12 * E2;
  d.zi11 = 2.0 * ys.zi12 * E2 - ys.Pp * E3 - b2;
  d.zr12 = ys.zr22 * E2 - ys.zr11 * md.inv_mass;
  d.zi12 = ys.zi22 * E2 - ys.zi11 * md.inv_mass;
  d.zr22 = -2.0 * ys.zr12 * md.inv_mass;
  d.zi22 = -2.0 * ys.zi12 * md.inv_mass;
  d.S = b0;
  d.Lam = 2.0 * fabs(v * k.d21);
#define SHGB_ODE2_FIELDS(F) F(q) F(p) F(Pq) F(Pp) F(zr11) F(zr12) F(zr22) F(zi11) F(zi12) F(zi22) F(S) F(Lam)
  if (stage == 0) {
#define F(f) acc.f = d.f; ys.f = y0.f + c * d.f;
    SHGB_ODE2_FIELDS(F)
#undef F
  } else if (stage < 3) {
#define F(f) acc.f = acc.f + 2.0 * d.f; ys.f = y0.f + c * d.f;
    SHGB_ODE2_FIELDS(F)
#undef F
  } else {
#define F(f) acc.f = y0.f + h6 * (acc.f + d.f);
    SHGB_ODE2_FIELDS(F)
#undef F
  }
#undef SHGB_ODE2_FIELDS
}

// One classical RK4 step of size h on the current component, into out.
__host__ __device__ inline void rk4_2(const DevModel &md, HopCtx &hc, Counters &cnt, const Ode2 &y, double h,
                                      Ode2 &out) {
  Ode2 ys = y;
  const double h6 = h * (1.0 / 6.0);
#pragma unroll
  for (int st = 0; st < 4; ++st) stage2(md, hc, cnt, y, ys, out, st, st == 2 ? h : 0.5 * h, h6);
}

// The derivative of the beam ODEs at stage values ys on the beam's
// component (the formulas of stage2); the first evaluation of a step
// completes a pending hop at ys, the state where it began.
__host__ __device__ inline Ode2 deriv2(const DevModel &md, HopCtx &hc, Counters &cnt, const Ode2 &ys, bool first) {
  const Q1 k = qcle_q1(md, ys.q);
  const double v = ys.p * md.inv_mass;
  if (first && hc.pending) {
    hop_choose(v * k.d21, hc.h, hc.gid, hc.seed, cnt, kTieRel);
    hc.pending = false;
  }
  const int l = hc.h.comp;
  const double sg = comp_sigma(l), bc = comp_bcoef(l);
  const double E1 = sg * k.s1, E2 = sg * k.s2, E3 = sg * k.s3;
  const double b0 = bc * k.s, b1 = bc * k.s1, b2 = bc * k.s2;
  Ode2 d;
  d.q = v;
  d.p = -E1;
  d.Pq = b1 + E2 * ys.Pp;
  d.Pp = -ys.Pq * md.inv_mass;
  d.zr11 = 2.0 * ys.zr12 * E2;
  d.zi11 = 2.0 * ys.zi12 * E2 - ys.Pp * E3 - b2;
  d.zr12 = ys.zr22 * E2 - ys.zr11 * md.inv_mass;
  d.zi12 = ys.zi22 * E2 - ys.zi11 * md.inv_mass;
  d.zr22 = -2.0 * ys.zr12 * md.inv_mass;
  d.zi22 = -2.0 * ys.zi12 * md.inv_mass;
  d.S = b0;
  d.Lam = 2.0 * fabs(v * k.d21);
  return d;
}

// One step of Kutta's third-order Runge-Kutta method (Sec. 2.4 integrates
// with a third-order method without naming it): k1 = f(y),
// k2 = f(y + h k1 / 2), k3 = f(y + h (2 k2 - k1)), y + h (k1 + 4 k2 + k3) / 6.
__host__ __device__ inline void rk3_2(const DevModel &md, HopCtx &hc, Counters &cnt, const Ode2 &y, double h,
                                      Ode2 &out) {
#define SHGB_ODE2_FIELDS(F) F(q) F(p) F(Pq) F(Pp) F(zr11) F(zr12) F(zr22) F(zi11) F(zi12) F(zi22) F(S) F(Lam)
  const Ode2 k1 = deriv2(md, hc, cnt, y, true);
  Ode2 ys;
  const double hh = 0.5 * h, h6 = h * (1.0 / 6.0);
#define F(f) ys.f = y.f + hh * k1.f;
  SHGB_ODE2_FIELDS(F)
#undef F
  const Ode2 k2 = deriv2(md, hc, cnt, ys, false);
#define F(f) ys.f = y.f + h * (2.0 * k2.f - k1.f);
  SHGB_ODE2_FIELDS(F)
#undef F
  const Ode2 k3 = deriv2(md, hc, cnt, ys, false);
#define F(f) out.f = y.f + h6 * (k1.f + 4.0 * k2.f + k3.f);
  SHGB_ODE2_FIELDS(F)
#undef F
#undef SHGB_ODE2_FIELDS
}

// Complete a hop still pending at the end of a call.
__host__ __device__ inline void hop_finish(const DevModel &md, HopCtx &hc, double q, double p, Counters &cnt,
                                           double tie_rel) {
  if (!hc.pending) return;
  const Q1 k = qcle_q1(md, q);
  hop_choose(p * md.inv_mass * k.d21, hc.h, hc.gid, hc.seed, cnt, tie_rel);
  hc.pending = false;
}

// One call of the interval algorithm (Sec. 2.4 steps 3-5) for one beam with
// the classical RK4 step (RK = 4) or Kutta's third-order step (RK = 3): a
// trial over the rest of the interval, the shortened step to the
// interpolated hop time, or, after a hop, a new trial on the new component.
// Returns true when the interval is complete.  Each lane runs its own
// sequence of calls, so a wave does not run extra passes for the shortened
// and remaining steps of one lane's hop while the others wait: a lane that
// completes an interval goes on with its next one.
template <int RK = 4>
__host__ __device__ inline bool interval2_call(const DevModel &md, Ode2 &y, HopCtx &hc, IvPos &iv, Counters &cnt) {
  Ode2 yn;
  if constexpr (RK == 3) rk3_2(md, hc, cnt, y, iv.hstep, yn);
  else rk4_2(md, hc, cnt, y, iv.hstep, yn);
  const double E = hc.h.E;
  if (!iv.partial) {
    const bool capped = iv.hops >= SHGB_HOP_CAP;
    if (!capped && fabs(yn.Lam - E) <= kTieRel * E) cnt.thr_ties++;
    if (capped || !(yn.Lam >= E)) {  // no hop in the rest of the interval
      if (capped) cnt.cap++;
      y = yn;
      return true;
    }
    iv.theta = (E <= y.Lam) ? 0.0 : (E - y.Lam) / (yn.Lam - y.Lam);
    if (iv.theta > 0.0 && iv.theta < 1.0) {
      iv.partial = true;
      iv.hstep = iv.theta * iv.rem;
      return false;
    }
    if (iv.theta >= 1.0) y = yn;  // hop exactly at the end; theta == 0: hop now
  } else {
    y = yn;
    iv.partial = false;
  }
  hop_start(hc, y.Lam);
  ++iv.hops;
  iv.rem = iv.rem * (1.0 - iv.theta);
  if (!(iv.rem > 0.0)) return true;
  iv.hstep = iv.rem;
  return false;
}

// All nsteps intervals of one beam: calls until the last interval is complete.
template <int RK = 4>
__host__ __device__ inline void intervals2(const DevModel &md, Ode2 &y, HopCtx &hc, int nsteps, double dt,
                                           Counters &cnt) {
  IvPos iv;
  iv_begin(iv, dt);
  for (int s = 0; s < nsteps;) {
    if (interval2_call<RK>(md, y, hc, iv, cnt)) {
      ++s;
      iv_begin(iv, dt);
    }
  }
}

// All nsteps intervals of beam b (one thread), FP64.
template <int RK = 4>
__device__ inline void m2_beam(const DevModel &md, double *__restrict__ tr, double *__restrict__ sc,
                               int32_t *__restrict__ comp, uint32_t *__restrict__ nhop, int64_t n, int64_t ld,
                               uint64_t gid0, int nsteps, double dt, uint64_t seed, int64_t b, Counters &cnt) {
  const Layout L(2, ld);
  if (b < n) {
    Ode2 y;
    y.q = tr[L.X(0) * ld + b];
    y.p = tr[L.X(1) * ld + b];
    y.Pq = tr[L.P(0) * ld + b];
    y.Pp = tr[L.P(1) * ld + b];
    y.zr11 = tr[L.Zre(0) * ld + b];
    y.zr12 = tr[L.Zre(1) * ld + b];
    y.zr22 = tr[L.Zre(2) * ld + b];
    y.zi11 = tr[L.Zim(0) * ld + b];
    y.zi12 = tr[L.Zim(1) * ld + b];
    y.zi22 = tr[L.Zim(2) * ld + b];
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
    intervals2<RK>(md, y, hc, nsteps, dt, cnt);
    hop_finish(md, hc, y.q, y.p, cnt, kTieRel);
    const double chk = y.q + y.p + y.Pq + y.Pp + y.zr11 + y.zr12 + y.zr22 + y.zi11 + y.zi12 +
                       y.zi22 + y.S + y.Lam + h.logw;
    if (!isfinite(chk)) cnt.nonfinite++;
    // The stores' addresses are formed here rather than kept from the loads
    // across the interval loop (which would hold 36 registers for them).
    asm volatile("" : "+v"(b));
    tr[L.X(0) * ld + b] = y.q;
    tr[L.X(1) * ld + b] = y.p;
    tr[L.P(0) * ld + b] = y.Pq;
    tr[L.P(1) * ld + b] = y.Pp;
    tr[L.Zre(0) * ld + b] = y.zr11;
    tr[L.Zre(1) * ld + b] = y.zr12;
    tr[L.Zre(2) * ld + b] = y.zr22;
    tr[L.Zim(0) * ld + b] = y.zi11;
    tr[L.Zim(1) * ld + b] = y.zi12;
    tr[L.Zim(2) * ld + b] = y.zi22;
    sc[kRowS * ld + b] = y.S;
    sc[kRowLam * ld + b] = y.Lam;
    sc[kRowLogw * ld + b] = h.logw;
    sc[kRowPhre * ld + b] = h.phre;
    sc[kRowPhim * ld + b] = h.phim;
    sc[kRowE * ld + b] = h.E;
    comp[b] = h.comp;
    nhop[b] = h.nhop;
  }
}

// Three waves per SIMD (167 registers, no spills; the store addresses are
// formed after the interval loop): the state moves through HBM exactly once
// each way.  Two waves per SIMD run as fast.
__global__ void __launch_bounds__(256)
step_m2_kernel(DevModel md, double *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
               uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, int nsteps,
               double dt, uint64_t seed, uint64_t *diag) {
  Counters cnt;
  m2_beam(md, tr, sc, comp, nhop, n, ld, gid0, nsteps, dt, seed, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
          cnt);
  flush_counters(cnt, diag);
}

// The same with Kutta's third-order step.
__global__ void __launch_bounds__(256)
step_m2_rk3_kernel(DevModel md, double *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
                   uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, int nsteps,
                   double dt, uint64_t seed, uint64_t *diag) {
  Counters cnt;
  m2_beam<3>(md, tr, sc, comp, nhop, n, ld, gid0, nsteps, dt, seed,
             (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cnt);
  flush_counters(cnt, diag);
}

// ---------------------------------------------------------------------------
// Mixed precision: the right-hand side of the ten trajectory values (X, P,
// Z) is evaluated in FP32 at FP32 stage values (formed from the FP32
// rounding of the step's start); each step's increment
// h/6 (k1 + 2k2 + 2k3 + k4) is formed in FP32 and added to an FP64 copy of
// the state that lives in registers for the whole call (adding small FP32
// increments to FP32 values would lose their low bits step after step).
// S and Lam are accumulated in FP64 (neither feeds back into the
// right-hand side, so their stage values are never formed); hop times,
// thresholds and the hop itself are FP64.  The state is rounded to FP32
// once, when the call stores it.

struct Traj2f {
  float q, p, Pq, Pp, zr11, zr12, zr22, zi11, zi12, zi22;
};

// one step's increment
struct Inc2m {
  Traj2f t;
  double S, Lam;
};

__host__ __device__ inline void stage2m(const QcleF &mf, HopCtx &hc, Counters &cnt, const Traj2f &y0, Traj2f &ys,
                                        Inc2m &acc, int stage, float c, float h6, double h6d) {
  const Q1f k = qcle_q1f(mf, ys.q);
  const float v = ys.p * mf.inv_mass;
  if (stage == 0 && hc.pending) {  // the coupling from the FP32 quantities; ties within 1e-5
    hop_choose((double)(v * k.d21), hc.h, hc.gid, hc.seed, cnt, kTieRelMixed);
    hc.pending = false;
  }
  const int l = hc.h.comp;
  const float sg = (float)comp_sigma(l), bc = (float)comp_bcoef(l);
  const float E1 = sg * k.s1, E2 = sg * k.s2, E3 = sg * k.s3;
  const float b1 = bc * k.s1, b2 = bc * k.s2;
  Traj2f d;
  d.q = v;
  d.p = -E1;
  d.Pq = b1 + E2 * ys.Pp;
  d.Pp = -ys.Pq * mf.inv_mass;
  d.zr11 = 2.0f * ys.zr12 * E2;
  d.zi11 = 2.0f * ys.zi12 * E2 - ys.Pp * E3 - b2;
  d.zr12 = ys.zr22 * E2 - ys.zr11 * mf.inv_mass;
  d.zi12 = ys.zi22 * E2 - ys.zi11 * mf.inv_mass;
  d.zr22 = -2.0f * ys.zr12 * mf.inv_mass;
  d.zi22 = -2.0f * ys.zi12 * mf.inv_mass;
  const double dS = (double)(bc * k.s);
  const double dLam = (double)(2.0f * fabsf(v * k.d21));
#define SHGB_TRAJ2_FIELDS(F) F(q) F(p) F(Pq) F(Pp) F(zr11) F(zr12) F(zr22) F(zi11) F(zi12) F(zi22)
  if (stage == 0) {
#define F(f) acc.t.f = d.f; ys.f = y0.f + c * d.f;
    SHGB_TRAJ2_FIELDS(F)
#undef F
    acc.S = dS;
    acc.Lam = dLam;
  } else if (stage < 3) {
#define F(f) acc.t.f = acc.t.f + 2.0f * d.f; ys.f = y0.f + c * d.f;
    SHGB_TRAJ2_FIELDS(F)
#undef F
    acc.S = acc.S + 2.0 * dS;
    acc.Lam = acc.Lam + 2.0 * dLam;
  } else {
#define F(f) acc.t.f = h6 * (acc.t.f + d.f);
    SHGB_TRAJ2_FIELDS(F)
#undef F
    acc.S = h6d * (acc.S + dS);
    acc.Lam = h6d * (acc.Lam + dLam);
  }
}

// The increment of one classical RK4 step of size h on component l.  The
// stage values are formed in FP32 from the FP32 rounding of the step's start.
__host__ __device__ inline void rk4_2m(const QcleF &mf, HopCtx &hc, Counters &cnt, const Ode2 &y, double h,
                                       Inc2m &inc) {
  Traj2f y0;
#define F(f) y0.f = (float)y.f;
  SHGB_TRAJ2_FIELDS(F)
#undef F
  Traj2f ys = y0;
  const double h6d = h * (1.0 / 6.0);
  const float h6 = (float)h6d, hf = (float)h;
#pragma unroll
  for (int st = 0; st < 4; ++st) stage2m(mf, hc, cnt, y0, ys, inc, st, st == 2 ? hf : 0.5f * hf, h6, h6d);
}

__host__ __device__ inline void add_inc2m(Ode2 &y, const Inc2m &inc) {
#define F(f) y.f = y.f + (double)inc.t.f;
  SHGB_TRAJ2_FIELDS(F)
#undef F
  y.S = y.S + inc.S;
  y.Lam = y.Lam + inc.Lam;
}

// One call of the interval algorithm of interval2_call on the mixed state.
__host__ __device__ inline bool interval2m_call(const QcleF &mf, Ode2 &y, HopCtx &hc, IvPos &iv, Counters &cnt) {
  Inc2m inc;
  rk4_2m(mf, hc, cnt, y, iv.hstep, inc);
  const double E = hc.h.E;
  if (!iv.partial) {
    const bool capped = iv.hops >= SHGB_HOP_CAP;
    const double lam_n = y.Lam + inc.Lam;
    if (!capped && fabs(lam_n - E) <= kTieRelMixed * E) cnt.thr_ties++;
    if (capped || !(lam_n >= E)) {
      if (capped) cnt.cap++;
      add_inc2m(y, inc);
      return true;
    }
    iv.theta = (E <= y.Lam) ? 0.0 : (E - y.Lam) / (lam_n - y.Lam);
    if (iv.theta > 0.0 && iv.theta < 1.0) {
      iv.partial = true;
      iv.hstep = iv.theta * iv.rem;
      return false;
    }
    if (iv.theta >= 1.0) add_inc2m(y, inc);
  } else {
    add_inc2m(y, inc);
    iv.partial = false;
  }
  hop_start(hc, y.Lam);
  ++iv.hops;
  iv.rem = iv.rem * (1.0 - iv.theta);
  if (!(iv.rem > 0.0)) return true;
  iv.hstep = iv.rem;
  return false;
}

__host__ __device__ inline void intervals2m(const QcleF &mf, Ode2 &y, HopCtx &hc, int nsteps, double dt,
                                            Counters &cnt) {
  IvPos iv;
  iv_begin(iv, dt);
  for (int s = 0; s < nsteps;) {
    if (interval2m_call(mf, y, hc, iv, cnt)) {
      ++s;
      iv_begin(iv, dt);
    }
  }
}
#undef SHGB_TRAJ2_FIELDS

// All nsteps intervals of beam b (one thread), mixed precision.
__device__ inline void m2m_beam(const DevModel &md, float *__restrict__ tr, double *__restrict__ sc,
                                int32_t *__restrict__ comp, uint32_t *__restrict__ nhop, int64_t n, int64_t ld,
                                uint64_t gid0, int nsteps, double dt, uint64_t seed, int64_t b, Counters &cnt) {
  const Layout L(2, ld);
  if (b < n) {
    const QcleF mf = qcle_f32(md);
    Ode2 y;
    y.q = tr[L.X(0) * ld + b];
    y.p = tr[L.X(1) * ld + b];
    y.Pq = tr[L.P(0) * ld + b];
    y.Pp = tr[L.P(1) * ld + b];
    y.zr11 = tr[L.Zre(0) * ld + b];
    y.zr12 = tr[L.Zre(1) * ld + b];
    y.zr22 = tr[L.Zre(2) * ld + b];
    y.zi11 = tr[L.Zim(0) * ld + b];
    y.zi12 = tr[L.Zim(1) * ld + b];
    y.zi22 = tr[L.Zim(2) * ld + b];
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
    intervals2m(mf, y, hc, nsteps, dt, cnt);
    if (hc.pending) {  // FP32 coupling at the stored (rounded) state, as inside the loop
      const Q1f k = qcle_q1f(mf, (float)y.q);
      hop_choose((double)((float)y.p * mf.inv_mass * k.d21), h, hc.gid, hc.seed, cnt, kTieRelMixed);
      hc.pending = false;
    }
    const double chk = y.q + y.p + y.Pq + y.Pp + y.zr11 + y.zr12 + y.zr22 + y.zi11 + y.zi12 + y.zi22 + y.S +
                       y.Lam + h.logw;
    if (!isfinite(chk)) cnt.nonfinite++;
    asm volatile("" : "+v"(b));  // store addresses formed here, as in m2_beam
    tr[L.X(0) * ld + b] = (float)y.q;
    tr[L.X(1) * ld + b] = (float)y.p;
    tr[L.P(0) * ld + b] = (float)y.Pq;
    tr[L.P(1) * ld + b] = (float)y.Pp;
    tr[L.Zre(0) * ld + b] = (float)y.zr11;
    tr[L.Zre(1) * ld + b] = (float)y.zr12;
    tr[L.Zre(2) * ld + b] = (float)y.zr22;
    tr[L.Zim(0) * ld + b] = (float)y.zi11;
    tr[L.Zim(1) * ld + b] = (float)y.zi12;
    tr[L.Zim(2) * ld + b] = (float)y.zi22;
    sc[kRowS * ld + b] = y.S;
    sc[kRowLam * ld + b] = y.Lam;
    sc[kRowLogw * ld + b] = h.logw;
    sc[kRowPhre * ld + b] = h.phre;
    sc[kRowPhim * ld + b] = h.phim;
    sc[kRowE * ld + b] = h.E;
    comp[b] = h.comp;
    nhop[b] = h.nhop;
  }
}

// Three waves per SIMD (148 registers, no spills): 4 % faster than two
// waves per SIMD when the store addresses were kept across the loop.
__global__ void __launch_bounds__(256)
step_m2_mixed_kernel(DevModel md, float *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
                     uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, int nsteps, double dt,
                     uint64_t seed, uint64_t *diag) {
  Counters cnt;
  m2m_beam(md, tr, sc, comp, nhop, n, ld, gid0, nsteps, dt, seed, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
           cnt);
  flush_counters(cnt, diag);
}

// Persistent form for a batch: each workgroup takes tiles of TPB beams from
// the queue until none is left; the tile decides the instance.
template <int TPB>
__global__ void __launch_bounds__(TPB)
step_m2_batched(const BatchItem *__restrict__ items, int n_items, int64_t total_tiles, int grab, int nsteps,
                double dt, unsigned long long *queue, uint64_t *diag) {
  Counters cnt;
  for (;;) {
    const int64_t t0 = batch_grab(queue, grab);
    if (t0 >= total_tiles) break;
    const int64_t t1 = t0 + grab < total_tiles ? t0 + grab : total_tiles;
    for (int64_t t = t0; t < t1; ++t) {
      const BatchItem &it = items[batch_find(items, n_items, t)];
      m2_beam(it.md, (double *)it.tr, it.sc, it.comp, it.nhop, it.n, it.ld, it.gid0, nsteps, dt, it.seed,
              (t - it.tile0) * TPB + threadIdx.x, cnt);
    }
  }
  flush_counters(cnt, diag);
}

template <int TPB>
__global__ void __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(3)))
step_m2_mixed_batched(const BatchItem *__restrict__ items, int n_items, int64_t total_tiles, int grab, int nsteps,
                      double dt, unsigned long long *queue, uint64_t *diag) {
  Counters cnt;
  for (;;) {
    const int64_t t0 = batch_grab(queue, grab);
    if (t0 >= total_tiles) break;
    const int64_t t1 = t0 + grab < total_tiles ? t0 + grab : total_tiles;
    for (int64_t t = t0; t < t1; ++t) {
      const BatchItem &it = items[batch_find(items, n_items, t)];
      m2m_beam(it.md, (float *)it.tr, it.sc, it.comp, it.nhop, it.n, it.ld, it.gid0, nsteps, dt, it.seed,
               (t - it.tile0) * TPB + threadIdx.x, cnt);
    }
  }
  flush_counters(cnt, diag);
}

// beams per tile of the batched m = 2 kernels
int m2_tile_beams(int wpb) { return 64 * wpb; }

hipError_t launch_step_m2_batched(bool mixed_state, int wpb, const BatchItem *items, int n_items, int64_t total_tiles,
                                  int grab, int blocks, int nsteps, double dt, unsigned long long *queue,
                                  uint64_t *diag, hipStream_t stream) {
#define SHGB_M2B(TPB)                                                                                         \
  if (mixed_state)                                                                                            \
    hipLaunchKernelGGL(step_m2_mixed_batched<TPB>, dim3(blocks), dim3(TPB), 0, stream, items, n_items,        \
                       total_tiles, grab, nsteps, dt, queue, diag);                                          \
  else                                                                                                        \
    hipLaunchKernelGGL(step_m2_batched<TPB>, dim3(blocks), dim3(TPB), 0, stream, items, n_items, total_tiles, \
                       grab, nsteps, dt, queue, diag);
  if (wpb == 2) {
    SHGB_M2B(128)
  } else {
    SHGB_M2B(256)
  }
#undef SHGB_M2B
  return hipGetLastError();
}

hipError_t launch_step_m2_rk3(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                              uint64_t *diag, hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (st.n_beams + threads - 1) / threads;
  hipLaunchKernelGGL(step_m2_rk3_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, md, st.f64,
                     scalar_block(st), st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed,
                     diag);
  return hipGetLastError();
}

hipError_t launch_step_m2(const DevModel &md, const shgb_state &st, int nsteps, double dt,
                          uint64_t seed, uint64_t *diag, hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (st.n_beams + threads - 1) / threads;
  double *sc = scalar_block(st);
  if (mixed(st))
    hipLaunchKernelGGL(step_m2_mixed_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, md, st.f32, sc,
                       st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed, diag);
  else
    hipLaunchKernelGGL(step_m2_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, md, st.f64, sc,
                       st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed, diag);
  return hipGetLastError();
}

}  // namespace shgb
