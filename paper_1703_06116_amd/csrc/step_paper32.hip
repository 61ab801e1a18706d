// Beam stepping for the nonlinear two-component system of Sec. 3.2,
// eq:ex2, x in R^2: one thread per beam, all intervals in registers,
// FP64.  In the form d_t u + alpha.grad u = (i/eps) beta u + gamma u,
// with u = x1 + x2, v = x1 - x2, r2 = |x|^2:
//   alpha_1 = -(sin u, cos v),  alpha_2 = -(sin v, cos u),
//   beta_1 = sin r2,            beta_2 = cos r2,
//   gamma = r2 [[-1, 5], [-5, -1/2]]   (row receives from column).
// Beam ODEs (Sec. 2.3, eq:shgb_odes) on component l:
//   X' = alpha_l, S' = beta_l, P' = grad beta_l - J^T P, A' = gamma_ll A,
//   Z' = -Z J - J^T Z + i (Hess(P.alpha_l) - Hess beta_l),
//   Lam' = sum_{j != l} |gamma_jl| = 5 r2,
// with J = d alpha_l / dx.  A hop from l goes to the other component and
// multiplies the phase by the sign of gamma_jl (-1 from 1 to 2, +1 back).
#include "device.h"

namespace shgb {

struct OdeP32 {
  double x1, x2, P1, P2, zr11, zr12, zr22, zi11, zi12, zi22, S, Are, Aim, Lam;
};

#define SHGB_ODEP32_FIELDS(F) \
  F(x1) F(x2) F(P1) F(P2) F(zr11) F(zr12) F(zr22) F(zi11) F(zi12) F(zi22) F(S) F(Are) F(Aim) F(Lam)

// |gamma_jl| / r2 by column l, and the rate integrand as the sum over all j
// minus the diagonal (the oracle's order of operations).
__host__ __device__ inline double p32_rate(int l, double r2) {
  const double g0 = (l == 0 ? 1.0 : 5.0) * r2, g1 = (l == 0 ? 5.0 : 0.5) * r2;  // |gamma_0l|, |gamma_1l|
  return (g0 + g1) - (l == 0 ? g0 : g1);
}

__host__ __device__ inline void rhs_p32(int l, const OdeP32 &y, OdeP32 &d) {
  const double x1 = y.x1, x2 = y.x2;
  const double u = x1 + x2, v = x1 - x2, r2 = x1 * x1 + x2 * x2;
  double su, cu, sv, cv, sr, cr;
  sincos(u, &su, &cu);
  sincos(v, &sv, &cv);
  sincos(r2, &sr, &cr);
  double J00, J01, J10, J11, H00, H01, H11, fb, hI, hX;
  if (l == 0) {
    d.x1 = -su;
    d.x2 = -cv;
    J00 = -cu; J01 = -cu; J10 = sv; J11 = -sv;
    // Hess(P.alpha_1) = P1 sin u [[1,1],[1,1]] + P2 cos v [[1,-1],[-1,1]]
    const double a = y.P1 * su, b = y.P2 * cv;
    H00 = a + b; H01 = a - b; H11 = a + b;
    d.S = sr;
    fb = 2.0 * cr;            // grad beta = fb x
    hI = 2.0 * cr;            // Hess beta = hI I + hX x x^T
    hX = -4.0 * sr;
  } else {
    d.x1 = -sv;
    d.x2 = -cu;
    J00 = -cv; J01 = cv; J10 = su; J11 = su;
    // Hess(P.alpha_2) = P1 sin v [[1,-1],[-1,1]] + P2 cos u [[1,1],[1,1]]
    const double a = y.P1 * sv, b = y.P2 * cu;
    H00 = a + b; H01 = b - a; H11 = a + b;
    d.S = cr;
    fb = -2.0 * sr;
    hI = -2.0 * sr;
    hX = -4.0 * cr;
  }
  d.P1 = fb * x1 - (J00 * y.P1 + J10 * y.P2);
  d.P2 = fb * x2 - (J01 * y.P1 + J11 * y.P2);
  const double B00 = H00 - (hI + hX * x1 * x1), B01 = H01 - hX * x1 * x2, B11 = H11 - (hI + hX * x2 * x2);
  // (Z J) for Re and Im of the symmetric Z; J^T Z = (Z J)^T
  const double r11 = y.zr11 * J00 + y.zr12 * J10, r12 = y.zr11 * J01 + y.zr12 * J11;
  const double r21 = y.zr12 * J00 + y.zr22 * J10, r22 = y.zr12 * J01 + y.zr22 * J11;
  const double i11 = y.zi11 * J00 + y.zi12 * J10, i12 = y.zi11 * J01 + y.zi12 * J11;
  const double i21 = y.zi12 * J00 + y.zi22 * J10, i22 = y.zi12 * J01 + y.zi22 * J11;
  d.zr11 = -(r11 + r11);
  d.zr12 = -(r12 + r21);
  d.zr22 = -(r22 + r22);
  d.zi11 = B00 - (i11 + i11);
  d.zi12 = B01 - (i12 + i21);
  d.zi22 = B11 - (i22 + i22);
  const double gll = (l == 0 ? -1.0 : -0.5) * r2;
  d.Are = gll * y.Are;
  d.Aim = gll * y.Aim;
  d.Lam = p32_rate(l, r2);
}

__host__ __device__ inline void rk4_p32(int l, const OdeP32 &y, double h, OdeP32 &out) {
  OdeP32 ys = y, d;
  const double h6 = h / 6.0;
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    rhs_p32(l, ys, d);
    const double c = st == 2 ? h : 0.5 * h;
    if (st == 0) {
#define F(f) out.f = d.f; ys.f = y.f + c * d.f;
      SHGB_ODEP32_FIELDS(F)
#undef F
    } else if (st < 3) {
#define F(f) out.f = out.f + 2.0 * d.f; ys.f = y.f + c * d.f;
      SHGB_ODEP32_FIELDS(F)
#undef F
    } else {
#define F(f) out.f = y.f + h6 * (out.f + d.f);
      SHGB_ODEP32_FIELDS(F)
#undef F
    }
  }
}

// Hop from component l at x (Sec. 2.4 step 5): the only destination is the
// other component; the draw still decides ties and supplies the threshold.
__host__ __device__ inline void hop_p32(double x1, double x2, HopScalars &h, uint64_t gid, uint64_t seed,
                                        Counters &cnt) {
  const double r2 = x1 * x1 + x2 * x2;
  // column l of gamma: l = 0: (-r2, -5 r2); l = 1: (5 r2, -r2/2)
  const double col0 = h.comp == 0 ? -1.0 * r2 : 5.0 * r2;
  const double col1 = h.comp == 0 ? -5.0 * r2 : -0.5 * r2;
  const double kappa_like[SHGB_NCOMP] = {col0, col1, 0.0, 0.0};
  const U64x4 w = draw(seed, gid, (uint64_t)h.nhop + 1u, kTagHop);
  const double U = u01(w.v[0]);
  const double Y = u01(w.v[1]);
  const int l = h.comp, j = 1 - l;
  const double R = fabs(kappa_like[j]);
  int dest = l;
  if (R > 0.0) {
    const double UR = U * R;
    if (fabs(UR - R) <= kTieRel * R) cnt.dest_ties++;
    dest = j;  // U R < R for every U in (0, 1); else the last positive rate, the same j
    if (kappa_like[dest] < 0.0) { h.phre = -h.phre; h.phim = -h.phim; }
  } else {
    cnt.zero_rate++;
  }
  h.comp = dest;
  h.nhop += 1u;
  h.E = -log(1.0 - Y);
  cnt.hops++;
}

// One call of the interval algorithm (Sec. 2.4 steps 3-5), as
// interval_lq_call; true when the interval is complete.
__host__ __device__ inline bool interval_p32_call(OdeP32 &y, HopScalars &h, IvPos &iv, uint64_t gid, uint64_t seed,
                                                  Counters &cnt) {
  OdeP32 yn;
  rk4_p32(h.comp, y, iv.hstep, yn);
  if (!iv.partial) {
    const bool capped = iv.hops >= SHGB_HOP_CAP;
    if (!capped && fabs(yn.Lam - h.E) <= kTieRel * h.E) cnt.thr_ties++;
    if (capped || !(yn.Lam >= h.E)) {
      if (capped) cnt.cap++;
      y = yn;
      return true;
    }
    iv.theta = (h.E <= y.Lam) ? 0.0 : (h.E - y.Lam) / (yn.Lam - y.Lam);
    if (iv.theta > 0.0 && iv.theta < 1.0) {
      iv.partial = true;
      iv.hstep = iv.theta * iv.rem;
      return false;
    }
    if (iv.theta >= 1.0) y = yn;
  } else {
    y = yn;
    iv.partial = false;
  }
  h.logw += y.Lam;
  y.Lam = 0.0;
  h.Lam = 0.0;
  hop_p32(y.x1, y.x2, h, gid, seed, cnt);
  ++iv.hops;
  iv.rem = iv.rem * (1.0 - iv.theta);
  if (!(iv.rem > 0.0)) return true;
  iv.hstep = iv.rem;
  return false;
}

__global__ void __launch_bounds__(256)
step_p32_kernel(double *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
                uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, int nsteps, double dt, uint64_t seed,
                uint64_t *diag) {
  const Layout L(2, ld);
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Counters cnt;
  if (b < n) {
    OdeP32 y;
    y.x1 = tr[L.X(0) * ld + b];
    y.x2 = tr[L.X(1) * ld + b];
    y.P1 = tr[L.P(0) * ld + b];
    y.P2 = tr[L.P(1) * ld + b];
    y.zr11 = tr[L.Zre(0) * ld + b];
    y.zr12 = tr[L.Zre(1) * ld + b];
    y.zr22 = tr[L.Zre(2) * ld + b];
    y.zi11 = tr[L.Zim(0) * ld + b];
    y.zi12 = tr[L.Zim(1) * ld + b];
    y.zi22 = tr[L.Zim(2) * ld + b];
    y.S = sc[kRowS * ld + b];
    y.Are = sc[kRowAre * ld + b];
    y.Aim = sc[kRowAim * ld + b];
    y.Lam = sc[kRowLam * ld + b];
    HopScalars h;
    h.logw = sc[kRowLogw * ld + b];
    h.phre = sc[kRowPhre * ld + b];
    h.phim = sc[kRowPhim * ld + b];
    h.E = sc[kRowE * ld + b];
    h.comp = comp[b];
    h.nhop = nhop[b];
    h.Lam = y.Lam;
    const uint64_t gid = gid0 + (uint64_t)b;
    IvPos iv;
    iv_begin(iv, dt);
    for (int s = 0; s < nsteps;) {
      if (interval_p32_call(y, h, iv, gid, seed, cnt)) {
        ++s;
        iv_begin(iv, dt);
      }
    }
    double chk = h.logw;
#define F(f) chk += y.f;
    SHGB_ODEP32_FIELDS(F)
#undef F
    if (!isfinite(chk)) cnt.nonfinite++;
    int64_t bs = b;
    asm volatile("" : "+v"(bs));  // store addresses formed after the interval loop
    tr[L.X(0) * ld + bs] = y.x1;
    tr[L.X(1) * ld + bs] = y.x2;
    tr[L.P(0) * ld + bs] = y.P1;
    tr[L.P(1) * ld + bs] = y.P2;
    tr[L.Zre(0) * ld + bs] = y.zr11;
    tr[L.Zre(1) * ld + bs] = y.zr12;
    tr[L.Zre(2) * ld + bs] = y.zr22;
    tr[L.Zim(0) * ld + bs] = y.zi11;
    tr[L.Zim(1) * ld + bs] = y.zi12;
    tr[L.Zim(2) * ld + bs] = y.zi22;
    sc[kRowS * ld + bs] = y.S;
    sc[kRowAre * ld + bs] = y.Are;
    sc[kRowAim * ld + bs] = y.Aim;
    sc[kRowLam * ld + bs] = y.Lam;
    sc[kRowLogw * ld + bs] = h.logw;
    sc[kRowPhre * ld + bs] = h.phre;
    sc[kRowPhim * ld + bs] = h.phim;
    sc[kRowE * ld + bs] = h.E;
    comp[bs] = h.comp;
    nhop[bs] = h.nhop;
  }
  flush_counters(cnt, diag);
}

__global__ void __launch_bounds__(256)
hop_p32_kernel(const double *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
               uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, const int32_t *__restrict__ idx,
               int64_t n_idx, uint64_t seed, uint64_t *diag) {
  const Layout L(2, ld);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Counters cnt;
  uint32_t bad = 0;
  if (t < n_idx) {
    const int64_t b = idx[t];
    if (b < 0 || b >= n) {
      bad = 1;
    } else {
      HopScalars h;
      h.logw = sc[kRowLogw * ld + b] + sc[kRowLam * ld + b];
      h.Lam = 0.0;
      h.phre = sc[kRowPhre * ld + b];
      h.phim = sc[kRowPhim * ld + b];
      h.E = sc[kRowE * ld + b];
      h.comp = comp[b];
      h.nhop = nhop[b];
      hop_p32(tr[L.X(0) * ld + b], tr[L.X(1) * ld + b], h, gid0 + (uint64_t)b, seed, cnt);
      sc[kRowLogw * ld + b] = h.logw;
      sc[kRowLam * ld + b] = 0.0;
      sc[kRowPhre * ld + b] = h.phre;
      sc[kRowPhim * ld + b] = h.phim;
      sc[kRowE * ld + b] = h.E;
      comp[b] = h.comp;
      nhop[b] = h.nhop;
    }
  }
  flush_counters(cnt, diag);
  if (diag) {
    uint32_t x = bad;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd((unsigned long long *)&diag[SHGB_DIAG_BAD_INDEX], (unsigned long long)x);
  }
}

hipError_t launch_step_p32(const shgb_state &st, int nsteps, double dt, uint64_t seed, uint64_t *diag,
                           hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (st.n_beams + threads - 1) / threads;
  hipLaunchKernelGGL(step_p32_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, st.f64, scalar_block(st),
                     st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed, diag);
  return hipGetLastError();
}

hipError_t launch_hop_p32(const shgb_state &st, const int32_t *idx, int64_t n_idx, uint64_t seed, uint64_t *diag,
                          hipStream_t stream) {
  if (n_idx == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (n_idx + threads - 1) / threads;
  hipLaunchKernelGGL(hop_p32_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, st.f64, scalar_block(st),
                     st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, idx, n_idx, seed, diag);
  return hipGetLastError();
}

}  // namespace shgb
