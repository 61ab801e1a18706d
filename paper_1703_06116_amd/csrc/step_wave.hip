// Beam stepping for the d-dimensional QCLE (phase space m = 2d > 2): a group
// of LPB lanes per beam (64/LPB beams per wavefront), all intervals in
// registers.
//
// Model (Sec. 3.3 with a harmonic bath): E_l(r) = Vb(r) + sigma_l s(q1),
// Vb = sum_{k>=1} (M w_k^2 q_k^2 / 2 + lam q1 q_k), so H = Hess E_l is an
// arrowhead matrix: H_00 = sigma s'', H_0k = H_k0 = lam, H_kk = M w_k^2.
// With J = [[0, I/M], [-H, 0]] the beam ODEs of Sec. 2.3 eq. (2.24) read, for
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
// c < m of the group owns X_c and P_c; the scalars (S, Lam, weights, the
// threshold and the component) are replicated over the group, so the hop
// logic (Sec. 2.4 steps 3-5) is uniform within a group.
#include "device.h"

namespace shgb {

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int D, int LPB>
struct PG {
  static constexpr int M = 2 * D;
  static constexpr int NGRP = D * (D + 1) / 2;          // pair groups a <= b
  static constexpr int NG = (NGRP + LPB - 1) / LPB;     // groups per lane
  static constexpr int G = 64 / LPB;                    // beams per wavefront
  static_assert(M <= LPB, "X and P need one lane per coordinate");
};

// One beam's exchange area.
template <int D>
struct PgLds {
  double rp_r[D][D], rp_i[D][D];   // Zrp
  double pp_r[D][D], pp_i[D][D];   // Zpp (both triangles)
  double rho_r[D], rho_i[D], chi_r[D], chi_i[D];
  double x[2 * D], p[2 * D];
};

// Values of one pair group: Zrr_ab, Zrp_ab, Zrp_ba, Zpp_ab (re, im).
struct Grp {
  double rr_r, rr_i, ab_r, ab_i, ba_r, ba_i, pp_r, pp_i;
};

template <int D, int LPB>
struct PgY {
  Grp g[PG<D, LPB>::NG];
  double x, p, S, Lam;
};

template <int D, int LPB>
struct PgCtx {
  int r;                         // lane within the beam's group
  int a[PG<D, LPB>::NG], b[PG<D, LPB>::NG];  // pair of each owned group, -1: none
  double ka[PG<D, LPB>::NG], kb[PG<D, LPB>::NG];  // M w^2 of the pair's bath indices (0 for index 0)
  double kc;                     // M w^2 of the lane's coordinate (X/P lanes)
};

template <int D, int LPB>
__device__ inline void pg_publish(const PgCtx<D, LPB> &cx, const PgY<D, LPB> &y, PgLds<D> &s) {
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e) {
    const int a = cx.a[e], b = cx.b[e];
    if (a >= 0) {
      s.rp_r[a][b] = y.g[e].ab_r;
      s.rp_i[a][b] = y.g[e].ab_i;
      s.rp_r[b][a] = y.g[e].ba_r;   // a == b: the same entry, written twice with one value
      s.rp_i[b][a] = y.g[e].ba_i;
      s.pp_r[a][b] = y.g[e].pp_r;
      s.pp_i[a][b] = y.g[e].pp_i;
      s.pp_r[b][a] = y.g[e].pp_r;
      s.pp_i[b][a] = y.g[e].pp_i;
    }
  }
  if (cx.r < 2 * D) { s.x[cx.r] = y.x; s.p[cx.r] = y.p; }
  wave_lds_sync();
  if (cx.r < D) {
    const int i = cx.r;
    double sr = 0.0, si = 0.0;
    for (int k = 1; k < D; ++k) { sr += s.rp_r[i][k]; si += s.rp_i[i][k]; }
    s.rho_r[i] = sr;
    s.rho_i[i] = si;
  } else if (cx.r < 2 * D) {
    const int j = cx.r - D;
    double sr = 0.0, si = 0.0;
    for (int k = 1; k < D; ++k) { sr += s.pp_r[k][j]; si += s.pp_i[k][j]; }
    s.chi_r[j] = sr;
    s.chi_i[j] = si;
  }
  wave_lds_sync();
}

// One Runge-Kutta stage for the lane's share of the state.  The stage values
// ys have been published to s; the derivative of each owned value is formed
// and folded at once into the accumulator and the next stage:
//   stage 0: acc = k;            ys = y0 + c k
//   stage 1, 2: acc += 2 k;      ys = y0 + c k
//   stage 3: acc = y0 + h6 (acc + k)   (the step's result)
template <int D, int LPB>
__device__ inline void pg_stage(const DevModel &md, int l, const PgCtx<D, LPB> &cx, const PgY<D, LPB> &y0,
                                PgY<D, LPB> &ys, PgY<D, LPB> &acc, int stage, double c, double h6,
                                const PgLds<D> &s) {
  const double q1 = s.x[0], p1 = s.x[D];
  const Q1 k = qcle_q1(md, q1);
  const double sg = comp_sigma(l), bc = comp_bcoef(l);
  const double H00 = sg * k.s2, lam = md.lam, im = md.inv_mass;
  const double B00 = -s.p[D] * sg * k.s3 - bc * k.s2;
  auto fold = [&](double &a, double &yv, double y0v, double d) {
    if (stage == 0) a = d;
    else if (stage < 3) a = a + 2.0 * d;
    else a = y0v + h6 * (a + d);
    if (stage < 3) yv = y0v + c * d;
  };
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e) {
    const int a = cx.a[e], b = cx.b[e];
    if (a >= 0) {
      const Grp v = ys.g[e];
      const double Ha = a == 0 ? H00 : cx.ka[e], Hb = b == 0 ? H00 : cx.kb[e];
      // Zrr_ab' = (Zrp H)_ab + (Zrp H)_ba
      double xr = v.ab_r * Hb, xi = v.ab_i * Hb;
      if (b > 0) { xr += lam * s.rp_r[a][0]; xi += lam * s.rp_i[a][0]; }
      else { xr += lam * s.rho_r[a]; xi += lam * s.rho_i[a]; }
      double tr = v.ba_r * Ha, ti = v.ba_i * Ha;
      if (a > 0) { tr += lam * s.rp_r[b][0]; ti += lam * s.rp_i[b][0]; }
      else { tr += lam * s.rho_r[b]; ti += lam * s.rho_i[b]; }
      const double drr_r = xr + tr;
      const double drr_i = (xi + ti) + ((a == 0 && b == 0) ? B00 : 0.0);
      // Zrp_ab' = (H Zpp)_ab - Zrr_ab / M,  Zrp_ba' = (H Zpp)_ba - Zrr_ba / M
      double ur = Ha * v.pp_r, ui = Ha * v.pp_i;
      if (a > 0) { ur += lam * s.pp_r[0][b]; ui += lam * s.pp_i[0][b]; }
      else { ur += lam * s.chi_r[b]; ui += lam * s.chi_i[b]; }
      double wr = Hb * v.pp_r, wi = Hb * v.pp_i;
      if (b > 0) { wr += lam * s.pp_r[0][a]; wi += lam * s.pp_i[0][a]; }
      else { wr += lam * s.chi_r[a]; wi += lam * s.chi_i[a]; }
      const double dab_r = ur - v.rr_r * im, dab_i = ui - v.rr_i * im;
      const double dba_r = wr - v.rr_r * im, dba_i = wi - v.rr_i * im;
      // Zpp_ab' = -(Zrp_ba + Zrp_ab) / M
      const double dpp_r = -(v.ba_r + v.ab_r) * im, dpp_i = -(v.ba_i + v.ab_i) * im;
      const Grp &g0 = y0.g[e];
      Grp &ga = acc.g[e], &gy = ys.g[e];
      fold(ga.rr_r, gy.rr_r, g0.rr_r, drr_r);
      fold(ga.rr_i, gy.rr_i, g0.rr_i, drr_i);
      fold(ga.ab_r, gy.ab_r, g0.ab_r, dab_r);
      fold(ga.ab_i, gy.ab_i, g0.ab_i, dab_i);
      fold(ga.ba_r, gy.ba_r, g0.ba_r, dba_r);
      fold(ga.ba_i, gy.ba_i, g0.ba_i, dba_i);
      fold(ga.pp_r, gy.pp_r, g0.pp_r, dpp_r);
      fold(ga.pp_i, gy.pp_i, g0.pp_i, dpp_i);
    }
  }
  const int cc = cx.r;
  double dx = 0.0, dp = 0.0;
  if (cc < D) {
    dx = s.x[D + cc] * im;
    if (cc == 0) {
      double sp = 0.0;
      for (int j = 1; j < D; ++j) sp += s.p[D + j];
      dp = bc * k.s1 + H00 * s.p[D] + lam * sp;
    } else {
      dp = cx.kc * s.p[D + cc] + lam * s.p[D];
    }
  } else if (cc < 2 * D) {
    const int kk = cc - D;
    if (kk == 0) {
      double sq = 0.0;
      for (int j = 1; j < D; ++j) sq += s.x[j];
      dx = -(lam * sq + sg * k.s1);
    } else {
      dx = -(cx.kc * s.x[kk] + lam * s.x[0]);
    }
    dp = -s.p[kk] * im;
  }
  fold(acc.x, ys.x, y0.x, dx);
  fold(acc.p, ys.p, y0.p, dp);
  fold(acc.S, ys.S, y0.S, bc * k.s);
  fold(acc.Lam, ys.Lam, y0.Lam, 2.0 * fabs(p1 * im * k.d21));
}

// One classical RK4 step of the group's beam on component l, into `out`;
// `s` is clobbered.
template <int D, int LPB>
__device__ inline void pg_rk4(const DevModel &md, int l, const PgCtx<D, LPB> &cx, const PgY<D, LPB> &y, double h,
                              PgY<D, LPB> &out, PgLds<D> &s) {
  PgY<D, LPB> ys = y;
  const double h6 = h / 6.0;
  const double cs[3] = {0.5 * h, 0.5 * h, h};
#pragma unroll 1
  for (int st = 0; st < 4; ++st) {
    pg_publish(cx, ys, s);
    pg_stage(md, l, cx, y, ys, out, st, st < 3 ? cs[st] : 0.0, h6, s);
    wave_lds_sync();
  }
}

template <int D, int LPB>
__device__ inline void pg_interval(const DevModel &md, const PgCtx<D, LPB> &cx, int base, PgY<D, LPB> &y,
                                   HopScalars &h, double dt, uint64_t gid, uint64_t seed, Counters &cnt,
                                   PgLds<D> &s) {
  double rem = dt, hstep = dt, theta = 1.0;
  bool partial = false;
  int hops = 0;
  PgY<D, LPB> yn;
  for (;;) {
    pg_rk4(md, h.comp, cx, y, hstep, yn, s);
    if (!partial) {
      const bool capped = hops >= SHGB_HOP_CAP;
      if (!capped && fabs(yn.Lam - h.E) <= kTieRel * h.E) cnt.thr_ties++;
      if (capped || !(yn.Lam >= h.E)) {
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
      if (theta >= 1.0) y = yn;
    } else {
      y = yn;
      partial = false;
    }
    h.Lam = y.Lam;
    const double q1 = __shfl(y.x, base, 64), p1 = __shfl(y.x, base + D, 64);
    hop_event(md, q1, p1, h, gid, seed, cnt);
    y.Lam = h.Lam;
    ++hops;
    rem = rem * (1.0 - theta);
    if (!(rem > 0.0)) break;
    hstep = rem;
  }
}

constexpr int kWavesPerBlock = 4;
#ifndef SHGB_D12_LANES_PER_BEAM
#define SHGB_D12_LANES_PER_BEAM 32
#endif
constexpr int kLanesPerBeamD12 = SHGB_D12_LANES_PER_BEAM;  // 32: two beams per wavefront

template <int D, int LPB>
__global__ void __launch_bounds__(64 * kWavesPerBlock)
step_wave_kernel(DevModel md, double *__restrict__ f, int32_t *__restrict__ comp, uint32_t *__restrict__ nhop,
                 int64_t n, int64_t ld, uint64_t gid0, int nsteps, double dt, uint64_t seed, uint64_t *diag) {
  using C = PG<D, LPB>;
  constexpr int M = C::M;
  __shared__ PgLds<D> lds[kWavesPerBlock * C::G];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = lane / LPB, r = lane % LPB, base = grp * LPB;
  const int slot = wid * C::G + grp;
  const int64_t b = (int64_t)blockIdx.x * (kWavesPerBlock * C::G) + slot;
  Counters cnt;
  if (b < n) {  // uniform across the beam's lanes
    const Layout L(M, ld);
    PgLds<D> &s = lds[slot];
    PgCtx<D, LPB> cx;
    cx.r = r;
    cx.kc = (r > 0 && r < D) ? md.bath_k[r] : ((r > D && r < M) ? md.bath_k[r - D] : 0.0);
    PgY<D, LPB> y;
#pragma unroll
    for (int e = 0; e < C::NG; ++e) {
      const int gi = r + LPB * e;
      cx.a[e] = cx.b[e] = -1;
      cx.ka[e] = cx.kb[e] = 0.0;
      y.g[e] = Grp{0, 0, 0, 0, 0, 0, 0, 0};
      if (gi < C::NGRP) {
        int a = 0, rem = gi;
        while (rem >= D - a) { rem -= D - a; ++a; }
        const int bb = a + rem;
        cx.a[e] = a;
        cx.b[e] = bb;
        cx.ka[e] = a > 0 ? md.bath_k[a] : 0.0;
        cx.kb[e] = bb > 0 ? md.bath_k[bb] : 0.0;
        const int trr = Layout::tri(M, a, bb), tab = Layout::tri(M, a, D + bb), tba = Layout::tri(M, bb, D + a),
                  tpp = Layout::tri(M, D + a, D + bb);
        y.g[e] = Grp{f[L.Zre(trr) * ld + b], f[L.Zim(trr) * ld + b], f[L.Zre(tab) * ld + b], f[L.Zim(tab) * ld + b],
                     f[L.Zre(tba) * ld + b], f[L.Zim(tba) * ld + b], f[L.Zre(tpp) * ld + b], f[L.Zim(tpp) * ld + b]};
      }
    }
    y.x = r < M ? f[L.X(r) * ld + b] : 0.0;
    y.p = r < M ? f[L.P(r) * ld + b] : 0.0;
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
    for (int st = 0; st < nsteps; ++st) pg_interval<D, LPB>(md, cx, base, y, h, dt, gid, seed, cnt, s);
    double chk = y.x + y.p + y.S + y.Lam + h.logw;
#pragma unroll
    for (int e = 0; e < C::NG; ++e) chk += y.g[e].rr_r + y.g[e].rr_i + y.g[e].ab_r + y.g[e].ab_i + y.g[e].ba_r +
                                            y.g[e].ba_i + y.g[e].pp_r + y.g[e].pp_i;
    int bad = !isfinite(chk);
#pragma unroll
    for (int off = 1; off < LPB; off <<= 1) bad |= __shfl_xor(bad, off, 64);
#pragma unroll
    for (int e = 0; e < C::NG; ++e) {
      const int a = cx.a[e], bb = cx.b[e];
      if (a >= 0) {
        const int trr = Layout::tri(M, a, bb), tab = Layout::tri(M, a, D + bb), tba = Layout::tri(M, bb, D + a),
                  tpp = Layout::tri(M, D + a, D + bb);
        f[L.Zre(trr) * ld + b] = y.g[e].rr_r;
        f[L.Zim(trr) * ld + b] = y.g[e].rr_i;
        f[L.Zre(tab) * ld + b] = y.g[e].ab_r;
        f[L.Zim(tab) * ld + b] = y.g[e].ab_i;
        if (a != bb) {
          f[L.Zre(tba) * ld + b] = y.g[e].ba_r;
          f[L.Zim(tba) * ld + b] = y.g[e].ba_i;
        }
        f[L.Zre(tpp) * ld + b] = y.g[e].pp_r;
        f[L.Zim(tpp) * ld + b] = y.g[e].pp_i;
      }
    }
    if (r < M) {
      f[L.X(r) * ld + b] = y.x;
      f[L.P(r) * ld + b] = y.p;
    }
    if (r == 0) {
      f[L.S() * ld + b] = y.S;
      f[L.Lam() * ld + b] = y.Lam;
      f[L.logw() * ld + b] = h.logw;
      f[L.phre() * ld + b] = h.phre;
      f[L.phim() * ld + b] = h.phim;
      f[L.E() * ld + b] = h.E;
      comp[b] = h.comp;
      nhop[b] = h.nhop;
      if (bad) cnt.nonfinite++;
    } else {
      cnt = Counters();  // the group's replicated counts are reported by its lane 0
    }
  }
  flush_counters(cnt, diag);
}

bool step_wave_supported(int d) { return d == 2 || d == 3 || d == 4 || d == 12; }

template <int D, int LPB>
static void launch_pg(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed, uint64_t *diag,
                      hipStream_t stream) {
  constexpr int beams_per_block = kWavesPerBlock * PG<D, LPB>::G;
  const int64_t blocks = (st.n_beams + beams_per_block - 1) / beams_per_block;
  hipLaunchKernelGGL((step_wave_kernel<D, LPB>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, stream, md,
                     st.f64, st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed, diag);
}

hipError_t launch_step_wave(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                            uint64_t *diag, hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  switch (md.d) {
    case 2: launch_pg<2, 8>(md, st, nsteps, dt, seed, diag, stream); break;
    case 3: launch_pg<3, 8>(md, st, nsteps, dt, seed, diag, stream); break;
    case 4: launch_pg<4, 8>(md, st, nsteps, dt, seed, diag, stream); break;
    case 12: launch_pg<12, kLanesPerBeamD12>(md, st, nsteps, dt, seed, diag, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace shgb
