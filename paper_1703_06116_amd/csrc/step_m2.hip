// Beam stepping for the one-dimensional QCLE (phase space m = 2): one thread
// per beam, the whole beam state in registers for all nsteps intervals.
//
// Beam ODEs (Sec. 2.3, eq. (2.24)) on component l, x = (q, p), v = p/M:
//   X' = alpha_l = (v, -E_l'),  J = d alpha_l / dx = [[0, 1/M], [-E_l'', 0]]
//   P' = grad beta_l - J^T P      = (beta_l' + E_l'' P_p, -P_q / M)
//   Z' = -Z J - J^T Z + i (Hess(P.alpha_l) - Hess beta_l),  Z = M + iN,
//        Hess(P.alpha_l) = [[-P_p E_l''', 0], [0, 0]]
//   S' = beta_l,  A' = gamma_ll A = 0,  Lam' = sum_{j != l} |gamma_jl| = 2 |v d21|
// The interval algorithm (Sec. 2.4 steps 3-5) runs one RK4 call site in a
// loop: a trial over the rest of the interval, then, if Lam crosses the
// threshold, the shortened step to the interpolated hop time, the hop, and a
// new trial on the new component.
#include "device.h"

namespace shgb {

struct Ode2 {
  double q, p, Pq, Pp, zr11, zr12, zr22, zi11, zi12, zi22, S, Lam;
};

__host__ __device__ inline Ode2 rhs2(const DevModel &md, int l, const Ode2 &y) {
  const Q1 k = qcle_q1(md, y.q);
  const double sg = comp_sigma(l), bc = comp_bcoef(l);
  const double v = y.p * md.inv_mass;
  const double E1 = sg * k.s1, E2 = sg * k.s2, E3 = sg * k.s3;
  const double b0 = bc * k.s, b1 = bc * k.s1, b2 = bc * k.s2;
  Ode2 d;
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

#define SHGB_ODE2_FIELDS(F) F(q) F(p) F(Pq) F(Pp) F(zr11) F(zr12) F(zr22) F(zi11) F(zi12) F(zi22) F(S) F(Lam)

__host__ __device__ inline Ode2 axpy2(const Ode2 &y, double h, const Ode2 &k) {
  Ode2 o;
#define F(f) o.f = y.f + h * k.f;
  SHGB_ODE2_FIELDS(F)
#undef F
  return o;
}

__host__ __device__ inline Ode2 rk4_2(const DevModel &md, int l, const Ode2 &y, double h) {
  const Ode2 k1 = rhs2(md, l, y);
  const Ode2 k2 = rhs2(md, l, axpy2(y, 0.5 * h, k1));
  const Ode2 k3 = rhs2(md, l, axpy2(y, 0.5 * h, k2));
  const Ode2 k4 = rhs2(md, l, axpy2(y, h, k3));
  const double h6 = h / 6.0;
  Ode2 o;
#define F(f) o.f = y.f + h6 * (k1.f + 2.0 * k2.f + 2.0 * k3.f + k4.f);
  SHGB_ODE2_FIELDS(F)
#undef F
  return o;
}

// One interval [t_n, t_n + dt] for one beam.
__host__ __device__ inline void interval2(const DevModel &md, Ode2 &y, HopScalars &h, double dt,
                                 uint64_t gid, uint64_t seed, Counters &cnt) {
  double rem = dt;      // time left in the interval
  double hstep = dt;    // size of the next RK4 call
  double theta = 1.0;
  bool partial = false; // the next call is the shortened step to the hop time
  int hops = 0;
  for (;;) {
    const Ode2 yn = rk4_2(md, h.comp, y, hstep);
    if (!partial) {
      const bool capped = hops >= SHGB_HOP_CAP;
      if (!capped && fabs(yn.Lam - h.E) <= kTieRel * h.E) cnt.thr_ties++;
      if (capped || !(yn.Lam >= h.E)) {  // no hop in the rest of the interval
        if (capped) cnt.cap++;
        y = yn;
        break;
      }
      theta = (h.E <= y.Lam) ? 0.0 : (h.E - y.Lam) / (yn.Lam - y.Lam);
      if (theta > 0.0 && theta < 1.0) {
        partial = true;
        hstep = theta * rem;
        continue;
      }
      if (theta >= 1.0) y = yn;  // hop exactly at the end; theta == 0: hop now
    } else {
      y = yn;
      partial = false;
    }
    h.Lam = y.Lam;
    hop_event(md, y.q, y.p, h, gid, seed, cnt);
    y.Lam = h.Lam;
    ++hops;
    rem = rem * (1.0 - theta);
    if (!(rem > 0.0)) break;
    hstep = rem;
  }
}

__global__ void __launch_bounds__(256)
step_m2_kernel(DevModel md, double *__restrict__ f, int32_t *__restrict__ comp,
               uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, int nsteps,
               double dt, uint64_t seed, uint64_t *diag) {
  const Layout L(2, ld);
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = b < n;
  Counters cnt;
  if (live) {
    Ode2 y;
    y.q = f[L.X(0) * ld + b];
    y.p = f[L.X(1) * ld + b];
    y.Pq = f[L.P(0) * ld + b];
    y.Pp = f[L.P(1) * ld + b];
    y.zr11 = f[L.Zre(0) * ld + b];
    y.zr12 = f[L.Zre(1) * ld + b];
    y.zr22 = f[L.Zre(2) * ld + b];
    y.zi11 = f[L.Zim(0) * ld + b];
    y.zi12 = f[L.Zim(1) * ld + b];
    y.zi22 = f[L.Zim(2) * ld + b];
    y.S = f[L.S() * ld + b];
    y.Lam = f[L.Lam() * ld + b];
    HopScalars h;
    h.logw = f[L.logw() * ld + b];
    h.phre = f[L.phre() * ld + b];
    h.phim = f[L.phim() * ld + b];
    h.E = f[L.E() * ld + b];
    h.comp = comp[b];
    h.nhop = nhop[b];
    h.Lam = y.Lam;
    const uint64_t gid = gid0 + (uint64_t)b;
    for (int s = 0; s < nsteps; ++s) interval2(md, y, h, dt, gid, seed, cnt);
    const double chk = y.q + y.p + y.Pq + y.Pp + y.zr11 + y.zr12 + y.zr22 + y.zi11 + y.zi12 +
                       y.zi22 + y.S + y.Lam + h.logw;
    if (!isfinite(chk)) cnt.nonfinite++;
    f[L.X(0) * ld + b] = y.q;
    f[L.X(1) * ld + b] = y.p;
    f[L.P(0) * ld + b] = y.Pq;
    f[L.P(1) * ld + b] = y.Pp;
    f[L.Zre(0) * ld + b] = y.zr11;
    f[L.Zre(1) * ld + b] = y.zr12;
    f[L.Zre(2) * ld + b] = y.zr22;
    f[L.Zim(0) * ld + b] = y.zi11;
    f[L.Zim(1) * ld + b] = y.zi12;
    f[L.Zim(2) * ld + b] = y.zi22;
    f[L.S() * ld + b] = y.S;
    f[L.Lam() * ld + b] = y.Lam;
    f[L.logw() * ld + b] = h.logw;
    f[L.phre() * ld + b] = h.phre;
    f[L.phim() * ld + b] = h.phim;
    f[L.E() * ld + b] = h.E;
    comp[b] = h.comp;
    nhop[b] = h.nhop;
  }
  flush_counters(cnt, diag);
}

hipError_t launch_step_m2(const DevModel &md, const shgb_state &st, int nsteps, double dt,
                          uint64_t seed, uint64_t *diag, hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (st.n_beams + threads - 1) / threads;
  hipLaunchKernelGGL(step_m2_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, md, st.f64,
                     st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed, diag);
  return hipGetLastError();
}

}  // namespace shgb
