// Pathwise derivative of the populations of the one-dimensional QCLE
// (m = 2) with respect to one model or initial-data parameter, by forward
// (tangent) propagation through the whole discrete algorithm.
//
// Every quantity of the stepping loop carries its value and its derivative
// along one direction theta_j of theta = (A, B, C, D, p_mean): the RK4
// stages of eq:shgb_odes, the hop time theta = (E - Lam)/(Lam' - Lam) and the
// shortened step it sets, the weight log w += Lam at each hop, and finally
// the closed-form beam integral c of Sec. 2.3 eq:shgb.  The discrete
// events are frozen at the values: every hop test, destination and phase
// sign is decided by the value part exactly as in the FP64 stepping kernel,
// and the thresholds E (drawn numbers) carry no derivative.  This is the
// derivative that central differences with common random numbers approach
// while no event flips.  p_mean shifts every initial p1, so its seed is
// dp1 = 1; A, B, C, D enter through the two-level quantities.
//
// One launch per direction keeps the dual state (value + derivative of the
// twelve integrated quantities, three RK4 copies) in registers.  The input
// state is read, never written.
#include "dual.h"

namespace shgb {

struct OdeDu {
  Du q, p, Pq, Pp, zr11, zr12, zr22, zi11, zi12, zi22, S, Lam;
};

#define SHGB_ODEDU_FIELDS(F) F(q) F(p) F(Pq) F(Pp) F(zr11) F(zr12) F(zr22) F(zi11) F(zi12) F(zi22) F(S) F(Lam)

__device__ inline void stage_du(const QcleDu &p, HopDu &hc, Counters &cnt, const OdeDu &y0, OdeDu &ys, OdeDu &acc,
                                int stage, Du c, Du h6) {
  const Q1Du k = qcle_q1_du(p, ys.q);
  const Du v = ys.p * p.inv_mass;
  if (stage == 0 && hc.pending) {  // frozen event: decided by the values
    hop_choose(v.v * k.d21.v, hc.h, hc.gid, hc.seed, cnt, kTieRel);
    hc.pending = false;
  }
  const int l = hc.h.comp;
  const double sg = comp_sigma(l), bc = comp_bcoef(l);
  const Du E1 = sg * k.s1, E2 = sg * k.s2, E3 = sg * k.s3;
  const Du b0 = bc * k.s, b1 = bc * k.s1, b2 = bc * k.s2;
  OdeDu d;
  d.q = v;
  d.p = -E1;
  d.Pq = b1 + E2 * ys.Pp;
  d.Pp = -(ys.Pq * p.inv_mass);
  d.zr11 = 2.0 * ys.zr12 * E2;
  d.zi11 = 2.0 * ys.zi12 * E2 - ys.Pp * E3 - b2;
  d.zr12 = ys.zr22 * E2 - ys.zr11 * p.inv_mass;
  d.zi12 = ys.zi22 * E2 - ys.zi11 * p.inv_mass;
  d.zr22 = -2.0 * ys.zr12 * p.inv_mass;
  d.zi22 = -2.0 * ys.zi12 * p.inv_mass;
  d.S = b0;
  d.Lam = 2.0 * dfabs(v * k.d21);
  if (stage == 0) {
#define F(f) acc.f = d.f; ys.f = y0.f + c * d.f;
    SHGB_ODEDU_FIELDS(F)
#undef F
  } else if (stage < 3) {
#define F(f) acc.f = acc.f + 2.0 * d.f; ys.f = y0.f + c * d.f;
    SHGB_ODEDU_FIELDS(F)
#undef F
  } else {
#define F(f) acc.f = y0.f + h6 * (acc.f + d.f);
    SHGB_ODEDU_FIELDS(F)
#undef F
  }
}

__device__ inline void rk4_du(const QcleDu &p, HopDu &hc, Counters &cnt, const OdeDu &y, Du h, OdeDu &out) {
  OdeDu ys = y;
  const Du h6 = h * (1.0 / 6.0);
  const Du hh = 0.5 * h;
#pragma unroll 1
  for (int st = 0; st < 4; ++st) stage_du(p, hc, cnt, y, ys, out, st, st == 2 ? h : hh, h6);
}

// One interval (Sec. 2.4 steps 3-5) on dual numbers; decisions by values.
__device__ inline void interval_du(const QcleDu &p, OdeDu &y, HopDu &hc, double dt, Counters &cnt) {
  Du rem = cst(dt), hstep = cst(dt), theta = cst(1.0);
  bool partial = false;
  int hops = 0;
  OdeDu yn;
  for (;;) {
    rk4_du(p, hc, cnt, y, hstep, yn);
    const double E = hc.h.E;
    if (!partial) {
      const bool capped = hops >= SHGB_HOP_CAP;
      if (!capped && fabs(yn.Lam.v - E) <= kTieRel * E) cnt.thr_ties++;
      if (capped || !(yn.Lam.v >= E)) {
        if (capped) cnt.cap++;
        y = yn;
        break;
      }
      // the hop time moves with the parameters: theta = (E - Lam)/(Lam' - Lam), E fixed
      theta = (E <= y.Lam.v) ? cst(0.0) : (cst(E) - y.Lam) / (yn.Lam - y.Lam);
      if (theta.v > 0.0 && theta.v < 1.0) {
        partial = true;
        hstep = theta * rem;
        continue;
      }
      if (theta.v >= 1.0) y = yn;
    } else {
      y = yn;
      partial = false;
    }
    hc.logw = hc.logw + y.Lam;
    y.Lam = cst(0.0);
    hc.pending = true;
    ++hops;
    rem = rem * (cst(1.0) - theta);
    if (!(rem.v > 0.0)) break;
    hstep = rem;
  }
}

constexpr int kTanThreads = 256;
constexpr int64_t kTanMaxBlocks = 2048;

__device__ inline void tan_block_store(const double (&acc)[kTanVals], double *out) {
  __shared__ double red[kTanThreads / 64][kTanVals];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kTanVals; ++k) {
    double s = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < kTanVals) {
    double s = 0.0;
    for (int w = 0; w < kTanThreads / 64; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// dir: 0..3 = A, B, C, D; 4 = p_mean.  Grid-stride over beams; block partial
// sums into partial[block][kTanVals].
__global__ void __launch_bounds__(kTanThreads)
tangent_m2_kernel(DevModel md, int dir, const double *__restrict__ tr, const double *__restrict__ sc,
                  const int32_t *__restrict__ comp, const uint32_t *__restrict__ nhop, int64_t n, int64_t ld,
                  uint64_t gid0, int nsteps, double dt, uint64_t seed, double *__restrict__ partial,
                  uint64_t *diag, int count_diag) {
  const Layout L(2, ld);
  QcleDu p;
  p.A = {md.A, dir == 0 ? 1.0 : 0.0};
  p.B = {md.B, dir == 1 ? 1.0 : 0.0};
  p.C = {md.C, dir == 2 ? 1.0 : 0.0};
  p.D = {md.D, dir == 3 ? 1.0 : 0.0};
  p.inv_mass = md.inv_mass;
  const double inv_eps = 1.0 / md.eps, norm = 2.0 * M_PI * md.eps;
  double acc[kTanVals];
#pragma unroll
  for (int k = 0; k < kTanVals; ++k) acc[k] = 0.0;
  Counters cnt;
  for (int64_t b = (int64_t)blockIdx.x * kTanThreads + threadIdx.x; b < n;
       b += (int64_t)gridDim.x * kTanThreads) {
    OdeDu y;
    y.q = cst(tr[L.X(0) * ld + b]);
    y.p = {tr[L.X(1) * ld + b], dir == 4 ? 1.0 : 0.0};
    y.Pq = cst(tr[L.P(0) * ld + b]);
    y.Pp = cst(tr[L.P(1) * ld + b]);
    y.zr11 = cst(tr[L.Zre(0) * ld + b]);
    y.zr12 = cst(tr[L.Zre(1) * ld + b]);
    y.zr22 = cst(tr[L.Zre(2) * ld + b]);
    y.zi11 = cst(tr[L.Zim(0) * ld + b]);
    y.zi12 = cst(tr[L.Zim(1) * ld + b]);
    y.zi22 = cst(tr[L.Zim(2) * ld + b]);
    y.S = cst(sc[kRowS * ld + b]);
    y.Lam = cst(sc[kRowLam * ld + b]);
    HopDu hc;
    hc.logw = cst(sc[kRowLogw * ld + b]);
    hc.h.logw = 0.0;
    hc.h.Lam = 0.0;
    hc.h.phre = sc[kRowPhre * ld + b];
    hc.h.phim = sc[kRowPhim * ld + b];
    hc.h.E = sc[kRowE * ld + b];
    hc.h.comp = comp[b];
    hc.h.nhop = nhop[b];
    hc.pending = false;
    hc.gid = gid0 + (uint64_t)b;
    hc.seed = seed;
    for (int s = 0; s < nsteps; ++s) interval_du(p, y, hc, dt, cnt);
    if (hc.pending) {
      const Q1Du k = qcle_q1_du(p, y.q);
      hop_choose(y.p.v * p.inv_mass * k.d21.v, hc.h, hc.gid, hc.seed, cnt, kTieRel);
      hc.pending = false;
    }
    // beam integral c = e^(logw + Lam) phase A e^(iS/eps) (2 pi eps) det(Z)^(-1/2) e^(-P^T Z^-1 P/(2 eps))
    const Cdu z11 = cd_of(y.zr11, y.zi11), z12 = cd_of(y.zr12, y.zi12), z22 = cd_of(y.zr22, y.zi22);
    const Cdu l21 = cd_div(z12, z11);
    const Cdu d2 = {csub(z22.v, cmul(l21.v, z12.v)), csub(z22.d, cadd(cmul(l21.d, z12.v), cmul(l21.v, z12.d)))};
    const Cdu P1 = cd_real(y.Pq);
    const Cdu w2 = {csub(cd_real(y.Pp).v, cmul(l21.v, P1.v)),
                    csub(cd_real(y.Pp).d, cadd(cmul(l21.d, P1.v), cmul(l21.v, P1.d)))};
    const Cdu quad1 = cd_div(cd_mul(P1, P1), z11), quad2 = cd_div(cd_mul(w2, w2), d2);
    const Cdu quad = {cadd(quad1.v, quad2.v), cadd(quad1.d, quad2.d)};
    const Cdu sq = cd_mul(cd_sqrt(z11), cd_sqrt(d2));
    const Cdu ex = cd_exp({cscale(quad.v, -0.5 * inv_eps), cscale(quad.d, -0.5 * inv_eps)});
    const Cdu g = cd_div(ex, sq);
    const Du mag = dexp(hc.logw + y.Lam);
    const Du ang = y.S * inv_eps;
    double sn, cs;
    sincos(ang.v, &sn, &cs);
    const cd pa = cmul({hc.h.phre, hc.h.phim}, {sc[kRowAre * ld + b], sc[kRowAim * ld + b]});
    const Cdu rot = {{cs, sn}, {-sn * ang.d, cs * ang.d}};
    const Cdu wgt = cd_mul({cscale(pa, mag.v), cscale(pa, mag.d)}, rot);
    const Cdu cb = cd_mul(wgt, g);
    const int l = hc.h.comp;
#pragma unroll
    for (int i = 0; i < SHGB_NCOMP; ++i) {
      const bool on = (l == i);
      acc[4 * i + 0] += on ? norm * cb.v.re : 0.0;
      acc[4 * i + 1] += on ? norm * cb.v.im : 0.0;
      acc[4 * i + 2] += on ? norm * cb.d.re : 0.0;
      acc[4 * i + 3] += on ? norm * cb.d.im : 0.0;
    }
    const double chk = y.q.v + y.p.v + y.zr11.v + y.zi11.v + y.S.v + hc.logw.v + y.q.d + y.p.d + y.zr11.d +
                       y.zi11.d + y.S.d + hc.logw.d;
    if (!isfinite(chk)) cnt.nonfinite++;
  }
  tan_block_store(acc, partial + (int64_t)blockIdx.x * kTanVals);
  if (count_diag) flush_counters(cnt, diag);  // once per call, not once per direction
}

__global__ void __launch_bounds__(kTanThreads)
tangent_final_kernel(const double *__restrict__ partial, int64_t nblocks, double *__restrict__ out) {
  double acc[kTanVals];
#pragma unroll
  for (int k = 0; k < kTanVals; ++k) acc[k] = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += kTanThreads)
#pragma unroll
    for (int k = 0; k < kTanVals; ++k) acc[k] += partial[b * kTanVals + k];
  tan_block_store(acc, out);
}

// Sum the per-block partials of one direction into out[kTanVals].
hipError_t launch_tangent_final(const double *partial, int64_t nblocks, double *out, hipStream_t stream) {
  hipLaunchKernelGGL(tangent_final_kernel, dim3(1), dim3(kTanThreads), 0, stream, partial, nblocks, out);
  return hipGetLastError();
}

int64_t tangent_blocks(int64_t n) {
  int64_t b = (n + kTanThreads - 1) / kTanThreads;
  if (b < 1) b = 1;
  return b < kTanMaxBlocks ? b : kTanMaxBlocks;
}

int64_t tangent_workspace_bytes(int64_t n) { return tangent_blocks(n) * kTanVals * (int64_t)sizeof(double); }

hipError_t launch_tangent_m2(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                             uint32_t dir_mask, double *out, void *work, uint64_t *diag, hipStream_t stream) {
  const int64_t blocks = tangent_blocks(st.n_beams);
  double *partial = (double *)work;
  int first = 1;
  for (int dir = 0; dir < 5; ++dir) {
    if (!(dir_mask & (1u << dir))) continue;
    hipLaunchKernelGGL(tangent_m2_kernel, dim3((unsigned)blocks), dim3(kTanThreads), 0, stream, md, dir, st.f64,
                       scalar_block(st), st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed,
                       partial, diag, first);
    first = 0;
    hipLaunchKernelGGL(tangent_final_kernel, dim3(1), dim3(kTanThreads), 0, stream, partial, blocks,
                       out + (int64_t)dir * kTanVals);
  }
  return hipGetLastError();
}

}  // namespace shgb
