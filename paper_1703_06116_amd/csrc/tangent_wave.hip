// Pathwise derivative of the populations of the d-dimensional QCLE with a
// harmonic bath (m = 2d > 2) with respect to theta = (A, B, C, D, p_mean):
// the contract of tangent_m2.hip (forward propagation of one direction per
// pass through the whole discrete algorithm, events frozen at the values,
// drawn thresholds without derivative) on the pair-group layout of the
// stepping kernel, here with one beam per wavefront.
//
// The stage values, the exchange area and the RK4 copies are dual numbers;
// the right-hand side is the stepping kernel's (grp_deriv, xp_deriv), the
// two-level quantities along q1 carry the derivative in A, B, C, D, and the
// hop time, the shortened step it sets and the weight update carry it as in
// the m = 2 pass.  After the last interval the beam's lanes assemble the
// dual Z and P in LDS and factor Z = L D L^T in dual complex arithmetic
// (no pivoting, as the populations kernel) for the beam integral
//   c = e^(logw + Lam) phase A e^(iS/eps) (2 pi eps)^(m/2) det(Z)^(-1/2)
//       e^(-P^T Z^-1 P / (2 eps)),
// whose value and derivative are summed per component.  The input state is
// read, never written.
#include "dual.h"
#include "wave.h"

namespace shgb {

constexpr int kTwLanes = 64;           // lanes per beam: one beam per wavefront
constexpr int kTwWaves = 2;            // beams per block
constexpr int64_t kTwMaxBlocks = 2048;

template <int D>
using PGW = PG<D, kTwLanes>;
static_assert(PG<12, kTwLanes>::NXP == 1, "one coordinate per lane");
template <int D>
using YW = PgY<D, kTwLanes, Du>;
template <int D>
using CtxW = PgCtx<D, kTwLanes, double>;

// Stage coefficients on dual numbers (a hop is completed where it starts,
// see pg_interval_du, as in the FP64 kernel).
template <int D>
__device__ inline StageCoef<Du> stage_coef_du(const QcleDu &p, int l, const PgLds<D, Du> &s, double lam) {
  StageCoef<Du> c;
  const Q1Du k = qcle_q1_du(p, s.x[0]);
  c.k = Q1T<Du>{k.s, k.s1, k.s2, k.s3, k.d21};
  c.im = Du(p.inv_mass);
  c.sg = Du(comp_sigma(l));
  c.bc = Du(comp_bcoef(l));
  c.H00 = c.sg * c.k.s2;
  c.lam = Du(lam);
  c.B00 = -s.p[D] * c.sg * c.k.s3 - c.bc * c.k.s2;
  return c;
}

// One RK4 stage (the fold of the FP64 stepping kernel) on dual numbers.
template <int D>
__device__ inline void pg_stage_du(const QcleDu &p, double lam, HopDu &hc, Counters &cnt, const CtxW<D> &cx,
                                   const YW<D> &y0, YW<D> &ys, YW<D> &acc, int stage, Du c, Du h6,
                                   const PgLds<D, Du> &s) {
  const StageCoef<Du> sc = stage_coef_du<D>(p, hc.h.comp, s, lam);
  auto fold = [&](Du &a, Du &yv, Du y0v, Du d) {
    if (stage == 0) a = d;
    else if (stage < 3) a = a + 2.0 * d;
    else a = y0v + h6 * (a + d);
    if (stage < 3) yv = y0v + c * d;
  };
#pragma unroll
  for (int e = 0; e < PGW<D>::NG; ++e) {
    if ((e + 1) * kTwLanes <= PGW<D>::NGRP || cx.a[e] >= 0) {   // slots every lane fills need no test
      Du d[kGrpN];
      grp_deriv<D, Du>(cx.a[e], cx.b[e], sc, ys.g[e].v, s, d);
#pragma unroll
      for (int j = 0; j < kGrpN; ++j) fold(acc.g[e].v[j], ys.g[e].v[j], y0.g[e].v[j], d[j]);
    }
  }
  Du dx, dp;
  xp_deriv<D, Du>(cx.r, sc, s, dx, dp);
  fold(acc.x[0], ys.x[0], y0.x[0], dx);
  fold(acc.p[0], ys.p[0], y0.p[0], dp);
  Du unused(0.0);
  fold(acc.S, unused, y0.S, sc.bc * sc.k.s);
  fold(acc.Lam, unused, y0.Lam, 2.0 * dfabs(s.x[D] * sc.im * sc.k.d21));
}

template <int D>
__device__ inline void pg_rk4_du(const QcleDu &p, double lam, HopDu &hc, Counters &cnt, const CtxW<D> &cx,
                                 const YW<D> &y, Du h, YW<D> &out, PgLds<D, Du> &s) {
  YW<D> ys = y;
  const Du h6 = h * (1.0 / 6.0);
  const Du hh = 0.5 * h;
#pragma unroll 1
  for (int st = 0; st < 4; ++st) {
    pg_publish(cx, ys, s);
    pg_stage_du<D>(p, lam, hc, cnt, cx, y, ys, out, st, st == 2 ? h : hh, h6, s);
    wave_lds_sync();
  }
}

// One interval (Sec. 2.4 steps 3-5), decisions by the values; the hop time
// theta = (E - Lam)/(Lam' - Lam) and the shortened step carry derivatives.
template <int D>
__device__ inline void pg_interval_du(const QcleDu &p, double lam, const CtxW<D> &cx, YW<D> &y, HopDu &hc,
                                      double dt, Counters &cnt, PgLds<D, Du> &s) {
  Du rem(dt), hstep(dt), theta(1.0);
  bool partial = false;
  int hops = 0;
  YW<D> yn;
  for (;;) {
    pg_rk4_du<D>(p, lam, hc, cnt, cx, y, hstep, yn, s);
    const double E = hc.h.E;
    if (!partial) {
      const bool capped = hops >= SHGB_HOP_CAP;
      if (!capped && fabs(yn.Lam.v - E) <= kTieRel * E) cnt.thr_ties++;
      if (capped || !(yn.Lam.v >= E)) {
        if (capped) cnt.cap++;
        y = yn;
        break;
      }
      theta = (E <= y.Lam.v) ? Du(0.0) : (Du(E) - y.Lam) / (yn.Lam - y.Lam);
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
    hc.logw = hc.logw + y.Lam;   // the hop: weight update, then the coupling at the state reached
    y.Lam = Du(0.0);
    {
      const Q1Du k = qcle_q1_du(p, Du(__shfl(y.x[0].v, 0, 64), __shfl(y.x[0].d, 0, 64)));
      hop_choose(__shfl(y.x[0].v, D, 64) * p.inv_mass * k.d21.v, hc.h, hc.gid, hc.seed, cnt, kTieRel);
    }
    ++hops;
    rem = rem * (Du(1.0) - theta);
    if (!(rem.v > 0.0)) break;
    hstep = rem;
  }
}

// The dual matrix Z (full, padded rows) and P of one beam for the factorisation.
template <int D>
struct TwFull {
  Cdu z[2 * D][2 * D + 1];
  Cdu w[2 * D];
};

template <int D>
union TwLds {
  PgLds<D, Du> ex;
  TwFull<D> f;
};

__device__ inline void tw_block_store(const double (&acc)[kTanVals], double *out) {
  __shared__ double red[kTwWaves][kTanVals];
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
    for (int w = 0; w < kTwWaves; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

__device__ inline Cdu cd_sub(Cdu a, Cdu b) { return {csub(a.v, b.v), csub(a.d, b.d)}; }
__device__ inline Cdu cd_add(Cdu a, Cdu b) { return {cadd(a.v, b.v), cadd(a.d, b.d)}; }

// dir: 0..3 = A, B, C, D; 4 = p_mean.  Wave-stride over beams (one beam per
// wavefront); block partial sums into partial[block][kTanVals].
template <int D>
__global__ void __launch_bounds__(64 * kTwWaves)
tangent_wave_kernel(DevModel md, int dir, const double *__restrict__ tr, const double *__restrict__ sc,
                    const int32_t *__restrict__ comp, const uint32_t *__restrict__ nhop, int64_t n, int64_t ld,
                    uint64_t gid0, int nsteps, double dt, uint64_t seed, double *__restrict__ partial,
                    uint64_t *diag, int count_diag) {
  constexpr int M = 2 * D;
  constexpr int NG = PGW<D>::NG;
  __shared__ TwLds<D> lds[kTwWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const Layout L(M, ld);
  QcleDu p;
  p.A = {md.A, dir == 0 ? 1.0 : 0.0};
  p.B = {md.B, dir == 1 ? 1.0 : 0.0};
  p.C = {md.C, dir == 2 ? 1.0 : 0.0};
  p.D = {md.D, dir == 3 ? 1.0 : 0.0};
  p.inv_mass = md.inv_mass;
  const double inv_eps = 1.0 / md.eps;
  const double pre = pow(2.0 * M_PI * md.eps, 0.5 * M);
  // the lane's pair groups and coordinate (the same for every beam)
  CtxW<D> cx;
  cx.r = lane;
  int rows[NG][kGrpN];
#pragma unroll
  for (int e = 0; e < NG; ++e) {
    const int gi = lane + kTwLanes * e;
    cx.a[e] = cx.b[e] = -1;
    if (gi < PGW<D>::NGRP) {
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
      for (int j = 0; j < kGrpN; ++j) rows[e][j] = row[j];
    }
  }
  double acc[kTanVals];
#pragma unroll
  for (int k = 0; k < kTanVals; ++k) acc[k] = 0.0;
  Counters cnt;
  for (int64_t b = (int64_t)blockIdx.x * kTwWaves + wid; b < n; b += (int64_t)gridDim.x * kTwWaves) {
    YW<D> y;
#pragma unroll
    for (int e = 0; e < NG; ++e)
#pragma unroll
      for (int j = 0; j < kGrpN; ++j) y.g[e].v[j] = Du(cx.a[e] >= 0 ? tr[rows[e][j] * ld + b] : 0.0);
    y.x[0] = Du(lane < M ? tr[L.X(lane) * ld + b] : 0.0, (dir == 4 && lane == D) ? 1.0 : 0.0);
    y.p[0] = Du(lane < M ? tr[L.P(lane) * ld + b] : 0.0);
    y.S = Du(sc[kRowS * ld + b]);
    y.Lam = Du(sc[kRowLam * ld + b]);
    HopDu hc;
    hc.logw = Du(sc[kRowLogw * ld + b]);
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
    pg_fill_const<D, kTwLanes>(lane, md.bath_k, lds[wid].ex);
    for (int st = 0; st < nsteps; ++st) pg_interval_du<D>(p, md.lam, cx, y, hc, dt, cnt, lds[wid].ex);
    double chk = y.S.v + y.S.d + y.Lam.v + y.Lam.d + hc.logw.v + hc.logw.d;
    if (lane < M) chk += y.x[0].v + y.x[0].d + y.p[0].v + y.p[0].d;
    // the beam integral: dual Z and P into LDS, then Z = L D L^T
    wave_lds_sync();
    TwFull<D> &f = lds[wid].f;
#pragma unroll
    for (int e = 0; e < NG; ++e) {
      const int a = cx.a[e], bb = cx.b[e];
      if (a >= 0) {
        const Du *v = y.g[e].v;
#pragma unroll
        for (int j = 0; j < kGrpN; ++j) chk += v[j].v + v[j].d;
        const Cdu rr = cd_of(v[kRrR], v[kRrI]), ab = cd_of(v[kAbR], v[kAbI]), ba = cd_of(v[kBaR], v[kBaI]),
                  pp = cd_of(v[kPpR], v[kPpI]);
        f.z[a][bb] = rr;
        f.z[bb][a] = rr;
        f.z[a][D + bb] = ab;          // Zrp_ab
        f.z[D + bb][a] = ab;
        f.z[D + a][D + bb] = pp;
        f.z[D + bb][D + a] = pp;
        if (a != bb) {
          f.z[bb][D + a] = ba;        // Zrp_ba
          f.z[D + a][bb] = ba;
        }
      }
    }
    if (lane < M) f.w[lane] = cd_real(y.p[0]);
    wave_lds_sync();
    Cdu sq = {{1.0, 0.0}, {0.0, 0.0}}, quad = {{0.0, 0.0}, {0.0, 0.0}};
    for (int k = 0; k < M; ++k) {
      const Cdu dk = f.z[k][k];
      const Cdu wk = f.w[k];
      sq = cd_mul(sq, cd_sqrt(dk));
      quad = cd_add(quad, cd_div(cd_mul(wk, wk), dk));
      // trailing update: Z_ij -= (Z_ik / d_k) Z_kj, w_i -= (Z_ik / d_k) w_k  (i, j > k)
      const int r = M - 1 - k;
      for (int t = lane; t < r * r; t += 64) {
        const int i = k + 1 + t / r, j = k + 1 + t % r;
        f.z[i][j] = cd_sub(f.z[i][j], cd_mul(cd_div(f.z[i][k], dk), f.z[k][j]));
      }
      if (lane < r) {
        const int i = k + 1 + lane;
        f.w[i] = cd_sub(f.w[i], cd_mul(cd_div(f.z[i][k], dk), wk));
      }
      wave_lds_sync();
    }
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
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < SHGB_NCOMP; ++i) {
        const bool on = (l == i);
        acc[4 * i + 0] += on ? pre * cb.v.re : 0.0;
        acc[4 * i + 1] += on ? pre * cb.v.im : 0.0;
        acc[4 * i + 2] += on ? pre * cb.d.re : 0.0;
        acc[4 * i + 3] += on ? pre * cb.d.im : 0.0;
      }
    }
    int bad = !isfinite(chk);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) bad |= __shfl_xor(bad, off, 64);
    if (bad && lane == 0) cnt.nonfinite++;
    wave_lds_sync();   // the exchange area is reused by the next beam
  }
  tw_block_store(acc, partial + (int64_t)blockIdx.x * kTanVals);
  if (count_diag) {
    if (lane != 0) cnt = Counters();   // the hop logic is replicated over the beam's lanes
    flush_counters(cnt, diag);
  }
}

int64_t tangent_wave_blocks(int64_t n) {
  int64_t b = (n + kTwWaves - 1) / kTwWaves;
  if (b < 1) b = 1;
  return b < kTwMaxBlocks ? b : kTwMaxBlocks;
}

int64_t tangent_wave_workspace_bytes(int64_t n) { return tangent_wave_blocks(n) * kTanVals * (int64_t)sizeof(double); }

bool tangent_wave_supported(int d) { return d == 2 || d == 3 || d == 4 || d == 12; }

hipError_t launch_tangent_final(const double *partial, int64_t nblocks, double *out, hipStream_t stream);

template <int D>
static hipError_t launch_tw(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                            uint32_t dir_mask, double *out, void *work, uint64_t *diag, hipStream_t stream) {
  const int64_t blocks = tangent_wave_blocks(st.n_beams);
  double *partial = (double *)work;
  int first = 1;
  for (int dir = 0; dir < SHGB_NTHETA; ++dir) {
    if (!(dir_mask & (1u << dir))) continue;
    hipLaunchKernelGGL(tangent_wave_kernel<D>, dim3((unsigned)blocks), dim3(64 * kTwWaves), 0, stream, md, dir,
                       st.f64, scalar_block(st), st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt,
                       seed, partial, diag, first);
    first = 0;
    const hipError_t e = launch_tangent_final(partial, blocks, out + (int64_t)dir * kTanVals, stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_tangent_wave(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                               uint32_t dir_mask, double *out, void *work, uint64_t *diag, hipStream_t stream) {
  switch (md.d) {
    case 2: return launch_tw<2>(md, st, nsteps, dt, seed, dir_mask, out, work, diag, stream);
    case 3: return launch_tw<3>(md, st, nsteps, dt, seed, dir_mask, out, work, diag, stream);
    case 4: return launch_tw<4>(md, st, nsteps, dt, seed, dir_mask, out, work, diag, stream);
    case 12: return launch_tw<12>(md, st, nsteps, dt, seed, dir_mask, out, work, diag, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace shgb
