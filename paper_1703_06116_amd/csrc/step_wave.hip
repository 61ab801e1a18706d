// Beam stepping for the d-dimensional QCLE (phase space m = 2d > 2): one
// wavefront per beam, all intervals in registers.
//
// Model (Sec. 3.3 with a harmonic bath): E_l(r) = Vb(r) + sigma_l s(q1),
// Vb = sum_{k>=1} (M w_k^2 q_k^2 / 2 + lam q1 q_k), so H = Hess E_l is an
// arrowhead matrix: H_00 = sigma s'', H_0k = H_k0 = lam, H_kk = M w_k^2.
// With J = [[0, I/M], [-H, 0]] the beam ODEs of Sec. 2.3 eq. (2.24) read, for
// Z = [[Zrr, Zrp], [Zrp^T, Zpp]] = M + iN,
//   Zrr' = Zrp H + (Zrp H)^T + i B,   B = e0 e0^T (-P_p0 sigma s''' - beta'' )
//   Zrp' = H Zpp - Zrr / M
//   Zpp' = -(Zrp + Zrp^T) / M
//   X'   = (p/M, -grad E_l),  P' = (grad_r beta + H P_p, -P_r / M),
//   S' = beta_l,  Lam' = 2 |v1 d21(q1)|
// and with the arrowhead H every product costs O(d^2):
//   (Zrp H)_ij = Zrp_ij H_jj + lam (j > 0 ? Zrp_i0 : sum_{k>0} Zrp_ik)
//   (H Zpp)_ij = H_ii Zpp_ij + lam (i > 0 ? Zpp_0j : sum_{k>0} Zpp_kj).
//
// Work split: lane t owns packed Z entries t, t+64, ... (upper triangle by
// rows), lane c < m owns X_c and P_c; the scalars S, Lam and the hop state
// are replicated in every lane, so the hop logic (Sec. 2.4 steps 3-5) is
// uniform across the wave.  Each RK4 stage publishes the stage Z, X, P to
// LDS (wave-private), forms the row/column sums, and every lane evaluates
// the derivatives of what it owns.
#include "device.h"

namespace shgb {

// Order the wave's LDS accesses: everything written before is visible to
// every lane of the wave after.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int D>
struct WaveCfg {
  static constexpr int M = 2 * D;
  static constexpr int T = M * (M + 1) / 2;
  static constexpr int NE = (T + 63) / 64;  // packed entries per lane
};

template <int D>
struct WaveLds {
  double zr[WaveCfg<D>::T], zi[WaveCfg<D>::T];
  double x[2 * D], p[2 * D];
  double rho_r[D], rho_i[D], chi_r[D], chi_i[D];
};

// Per-lane slice of the beam state.
template <int D>
struct WaveY {
  double zr[WaveCfg<D>::NE], zi[WaveCfg<D>::NE];
  double x, p;     // X_c, P_c for lane c < m
  double S, Lam;   // replicated
};

template <int D>
struct WaveCtx {
  int lane;
  int ea[WaveCfg<D>::NE], eb[WaveCfg<D>::NE];  // full indices (a <= b) of owned entries; -1: none
};

__device__ inline int tri_idx(int m, int a, int b) {
  return a <= b ? Layout::tri(m, a, b) : Layout::tri(m, b, a);
}

// Derivative of the lane's slice at the stage published in `s`.
template <int D>
__device__ inline WaveY<D> rhs_wave(const DevModel &md, int l, const WaveCtx<D> &cx, const WaveLds<D> &s) {
  constexpr int M = 2 * D;
  const double q1 = s.x[0], p1 = s.x[D];
  const Q1 k = qcle_q1(md, q1);
  const double sg = comp_sigma(l), bc = comp_bcoef(l);
  const double H00 = sg * k.s2, lam = md.lam, im = md.inv_mass;
  WaveY<D> d;
#pragma unroll
  for (int e = 0; e < WaveCfg<D>::NE; ++e) {
    const int a = cx.ea[e], b = cx.eb[e];
    double rr = 0.0, ri = 0.0;
    if (a >= 0) {
      if (b < D) {
        // Zrr entry (a, b): (Zrp H)_ab + (Zrp H)_ba  (+ i B at (0, 0))
        const int ab = tri_idx(M, a, D + b), ba = tri_idx(M, b, D + a);
        const double Hbb = b == 0 ? H00 : md.bath_k[b], Haa = a == 0 ? H00 : md.bath_k[a];
        double tr = s.zr[ab] * Hbb, ti = s.zi[ab] * Hbb;
        if (b > 0) { const int t0 = tri_idx(M, a, D); tr += lam * s.zr[t0]; ti += lam * s.zi[t0]; }
        else { tr += lam * s.rho_r[a]; ti += lam * s.rho_i[a]; }
        tr += s.zr[ba] * Haa;
        ti += s.zi[ba] * Haa;
        if (a > 0) { const int t0 = tri_idx(M, b, D); tr += lam * s.zr[t0]; ti += lam * s.zi[t0]; }
        else { tr += lam * s.rho_r[b]; ti += lam * s.rho_i[b]; }
        if (a == 0 && b == 0) ti += -s.p[D] * sg * k.s3 - bc * k.s2;
        rr = tr;
        ri = ti;
      } else if (a < D) {
        // Zrp entry (i, j) = (a, b - D): (H Zpp)_ij - Zrr_ij / M
        const int i = a, j = b - D;
        const double Hii = i == 0 ? H00 : md.bath_k[i];
        const int pp = tri_idx(M, D + i, D + j);
        double tr = Hii * s.zr[pp], ti = Hii * s.zi[pp];
        if (i > 0) { const int t0 = tri_idx(M, D, D + j); tr += lam * s.zr[t0]; ti += lam * s.zi[t0]; }
        else { tr += lam * s.chi_r[j]; ti += lam * s.chi_i[j]; }
        const int rrij = tri_idx(M, i, j);
        rr = tr - s.zr[rrij] * im;
        ri = ti - s.zi[rrij] * im;
      } else {
        // Zpp entry (i, j) = (a - D, b - D): -(Zrp_ji + Zrp_ij) / M
        const int i = a - D, j = b - D;
        const int ji = tri_idx(M, j, D + i), ij = tri_idx(M, i, D + j);
        rr = -(s.zr[ji] + s.zr[ij]) * im;
        ri = -(s.zi[ji] + s.zi[ij]) * im;
      }
    }
    d.zr[e] = rr;
    d.zi[e] = ri;
  }
  // X_c and P_c
  const int c = cx.lane;
  double dx = 0.0, dp = 0.0;
  if (c < D) {
    dx = s.x[D + c] * im;
    if (c == 0) {
      double sp = 0.0;
      for (int j = 1; j < D; ++j) sp += s.p[D + j];
      dp = bc * k.s1 + H00 * s.p[D] + lam * sp;
    } else {
      dp = md.bath_k[c] * s.p[D + c] + lam * s.p[D];
    }
  } else if (c < M) {
    const int kk = c - D;
    if (kk == 0) {
      double sq = 0.0;
      for (int j = 1; j < D; ++j) sq += s.x[j];
      dx = -(lam * sq + sg * k.s1);
    } else {
      dx = -(md.bath_k[kk] * s.x[kk] + lam * s.x[0]);
    }
    dp = -s.p[kk] * im;
  }
  d.x = dx;
  d.p = dp;
  d.S = bc * k.s;
  d.Lam = 2.0 * fabs(p1 * im * k.d21);
  return d;
}

template <int D>
__device__ inline void publish(const WaveCtx<D> &cx, const WaveY<D> &y, WaveLds<D> &s) {
  constexpr int M = 2 * D;
#pragma unroll
  for (int e = 0; e < WaveCfg<D>::NE; ++e) {
    const int t = cx.lane + 64 * e;
    if (t < WaveCfg<D>::T) { s.zr[t] = y.zr[e]; s.zi[t] = y.zi[e]; }
  }
  if (cx.lane < M) { s.x[cx.lane] = y.x; s.p[cx.lane] = y.p; }
  wave_lds_sync();
  // row sums of Zrp (lanes 0..D-1) and column sums of Zpp (lanes D..2D-1) over k > 0
  if (cx.lane < D) {
    const int i = cx.lane;
    double r = 0.0, im = 0.0;
    for (int k = 1; k < D; ++k) { const int t = tri_idx(M, i, D + k); r += s.zr[t]; im += s.zi[t]; }
    s.rho_r[i] = r;
    s.rho_i[i] = im;
  } else if (cx.lane < M) {
    const int j = cx.lane - D;
    double r = 0.0, im = 0.0;
    for (int k = 1; k < D; ++k) { const int t = tri_idx(M, D + k, D + j); r += s.zr[t]; im += s.zi[t]; }
    s.chi_r[j] = r;
    s.chi_i[j] = im;
  }
  wave_lds_sync();
}

template <int D>
__device__ inline void axpy_wave(WaveY<D> &o, const WaveY<D> &y, double h, const WaveY<D> &k) {
#pragma unroll
  for (int e = 0; e < WaveCfg<D>::NE; ++e) { o.zr[e] = y.zr[e] + h * k.zr[e]; o.zi[e] = y.zi[e] + h * k.zi[e]; }
  o.x = y.x + h * k.x;
  o.p = y.p + h * k.p;
  o.S = y.S + h * k.S;
  o.Lam = y.Lam + h * k.Lam;
}

// One classical RK4 step on component l; LDS `s` is clobbered.
template <int D>
__device__ inline WaveY<D> rk4_wave(const DevModel &md, int l, const WaveCtx<D> &cx, const WaveY<D> &y, double h,
                                    WaveLds<D> &s) {
  WaveY<D> acc, ys;
  publish(cx, y, s);
  WaveY<D> k = rhs_wave(md, l, cx, s);
  acc = k;
  wave_lds_sync();
  axpy_wave(ys, y, 0.5 * h, k);
  publish(cx, ys, s);
  k = rhs_wave(md, l, cx, s);
  axpy_wave(acc, acc, 2.0, k);
  wave_lds_sync();
  axpy_wave(ys, y, 0.5 * h, k);
  publish(cx, ys, s);
  k = rhs_wave(md, l, cx, s);
  axpy_wave(acc, acc, 2.0, k);
  wave_lds_sync();
  axpy_wave(ys, y, h, k);
  publish(cx, ys, s);
  k = rhs_wave(md, l, cx, s);
  wave_lds_sync();
  const double h6 = h / 6.0;
  WaveY<D> o;
#pragma unroll
  for (int e = 0; e < WaveCfg<D>::NE; ++e) {
    o.zr[e] = y.zr[e] + h6 * (acc.zr[e] + k.zr[e]);
    o.zi[e] = y.zi[e] + h6 * (acc.zi[e] + k.zi[e]);
  }
  o.x = y.x + h6 * (acc.x + k.x);
  o.p = y.p + h6 * (acc.p + k.p);
  o.S = y.S + h6 * (acc.S + k.S);
  o.Lam = y.Lam + h6 * (acc.Lam + k.Lam);
  return o;
}

template <int D>
__device__ inline void interval_wave(const DevModel &md, const WaveCtx<D> &cx, WaveY<D> &y, HopScalars &h,
                                     double dt, uint64_t gid, uint64_t seed, Counters &cnt, WaveLds<D> &s) {
  double rem = dt, hstep = dt, theta = 1.0;
  bool partial = false;
  int hops = 0;
  for (;;) {
    const WaveY<D> yn = rk4_wave(md, h.comp, cx, y, hstep, s);
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
    const double q1 = __shfl(y.x, 0, 64), p1 = __shfl(y.x, D, 64);
    hop_event(md, q1, p1, h, gid, seed, cnt);
    y.Lam = h.Lam;
    ++hops;
    rem = rem * (1.0 - theta);
    if (!(rem > 0.0)) break;
    hstep = rem;
  }
}

constexpr int kWavesPerBlock = 4;

template <int D>
__global__ void __launch_bounds__(64 * kWavesPerBlock)
step_wave_kernel(DevModel md, double *__restrict__ f, int32_t *__restrict__ comp, uint32_t *__restrict__ nhop,
                 int64_t n, int64_t ld, uint64_t gid0, int nsteps, double dt, uint64_t seed, uint64_t *diag) {
  constexpr int M = 2 * D;
  __shared__ WaveLds<D> lds[kWavesPerBlock];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  Counters cnt;
  if (b < n) {  // uniform across the wave
    const Layout L(M, ld);
    WaveLds<D> &s = lds[wid];
    WaveCtx<D> cx;
    cx.lane = lane;
    WaveY<D> y;
#pragma unroll
    for (int e = 0; e < WaveCfg<D>::NE; ++e) {
      const int t = lane + 64 * e;
      cx.ea[e] = cx.eb[e] = -1;
      y.zr[e] = y.zi[e] = 0.0;
      if (t < WaveCfg<D>::T) {
        int a = 0, rem = t;
        while (rem >= M - a) { rem -= M - a; ++a; }
        cx.ea[e] = a;
        cx.eb[e] = a + rem;
        y.zr[e] = f[L.Zre(t) * ld + b];
        y.zi[e] = f[L.Zim(t) * ld + b];
      }
    }
    y.x = lane < M ? f[L.X(lane) * ld + b] : 0.0;
    y.p = lane < M ? f[L.P(lane) * ld + b] : 0.0;
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
    for (int st = 0; st < nsteps; ++st) interval_wave<D>(md, cx, y, h, dt, gid, seed, cnt, s);
    // every lane checks its slice; the wave counts the beam once
    double chk = y.x + y.p + y.S + y.Lam + h.logw;
#pragma unroll
    for (int e = 0; e < WaveCfg<D>::NE; ++e) chk += y.zr[e] + y.zi[e];
    const bool bad = __any(!isfinite(chk));
#pragma unroll
    for (int e = 0; e < WaveCfg<D>::NE; ++e) {
      const int t = lane + 64 * e;
      if (t < WaveCfg<D>::T) {
        f[L.Zre(t) * ld + b] = y.zr[e];
        f[L.Zim(t) * ld + b] = y.zi[e];
      }
    }
    if (lane < M) {
      f[L.X(lane) * ld + b] = y.x;
      f[L.P(lane) * ld + b] = y.p;
    }
    if (lane == 0) {
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
      cnt = Counters();  // the replicated counts are reported by lane 0 only
    }
  }
  flush_counters(cnt, diag);
}

bool step_wave_supported(int d) { return d == 2 || d == 3 || d == 4 || d == 12; }

hipError_t launch_step_wave(const DevModel &md, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                            uint64_t *diag, hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  const int64_t blocks = (st.n_beams + kWavesPerBlock - 1) / kWavesPerBlock;
#define SHGB_STEP_CASE(DD)                                                                                  \
  case DD:                                                                                                  \
    hipLaunchKernelGGL(step_wave_kernel<DD>, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, stream, md, \
                       st.f64, st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed, diag); \
    break;
  switch (md.d) {
    SHGB_STEP_CASE(2)
    SHGB_STEP_CASE(3)
    SHGB_STEP_CASE(4)
    SHGB_STEP_CASE(12)
    default:
      return hipErrorInvalidValue;
  }
#undef SHGB_STEP_CASE
  return hipGetLastError();
}

}  // namespace shgb
