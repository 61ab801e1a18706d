// Beam stepping and hops for linear-quadratic systems (m = 2): one thread
// per beam, all intervals in registers, FP64.
//
// Beam ODEs (Sec. 2.3, eq:shgb_odes) on component l with alpha = a + J x,
// beta = b0 + b.x + x^T H x / 2 and constant gamma:
//   X' = a + J X,                 S' = beta(X),
//   P' = grad beta - J^T P = b + H X - J^T P,
//   Z' = -Z J - J^T Z - i H       (Hess(P.alpha) = 0 for linear alpha),
//   A' = gamma_ll A,              Lam' = sum_{j != l} |gamma_jl|.
// The interval algorithm (Sec. 2.4 steps 3-5) is the one of the QCLE
// kernels; the hop needs no coupling evaluation (gamma is constant).
#include "device.h"

namespace shgb {

struct OdeLQ {
  double x1, x2, P1, P2, zr11, zr12, zr22, zi11, zi12, zi22, S, Are, Aim, Lam;
};

#define SHGB_ODELQ_FIELDS(F) \
  F(x1) F(x2) F(P1) F(P2) F(zr11) F(zr12) F(zr22) F(zi11) F(zi12) F(zi22) F(S) F(Are) F(Aim) F(Lam)

__host__ __device__ inline void rhs_lq(const DevLQ &lq, int l, const OdeLQ &y, OdeLQ &d) {
  const double(&J)[2][2] = lq.J[l];
  const double(&H)[2][2] = lq.H[l];
  const double x1 = y.x1, x2 = y.x2;
  d.x1 = lq.a[l][0] + (J[0][0] * x1 + J[0][1] * x2);
  d.x2 = lq.a[l][1] + (J[1][0] * x1 + J[1][1] * x2);
  const double Hx1 = H[0][0] * x1 + H[0][1] * x2, Hx2 = H[1][0] * x1 + H[1][1] * x2;
  d.S = lq.b0[l] + (lq.b[l][0] * x1 + lq.b[l][1] * x2) + 0.5 * (x1 * Hx1 + x2 * Hx2);
  d.P1 = lq.b[l][0] + Hx1 - (J[0][0] * y.P1 + J[1][0] * y.P2);
  d.P2 = lq.b[l][1] + Hx2 - (J[0][1] * y.P1 + J[1][1] * y.P2);
  // (Z J) for the real and imaginary parts of the symmetric Z; (J^T Z) = (Z J)^T
  const double r11 = y.zr11 * J[0][0] + y.zr12 * J[1][0], r12 = y.zr11 * J[0][1] + y.zr12 * J[1][1];
  const double r21 = y.zr12 * J[0][0] + y.zr22 * J[1][0], r22 = y.zr12 * J[0][1] + y.zr22 * J[1][1];
  const double i11 = y.zi11 * J[0][0] + y.zi12 * J[1][0], i12 = y.zi11 * J[0][1] + y.zi12 * J[1][1];
  const double i21 = y.zi12 * J[0][0] + y.zi22 * J[1][0], i22 = y.zi12 * J[0][1] + y.zi22 * J[1][1];
  d.zr11 = -(r11 + r11);
  d.zr12 = -(r12 + r21);
  d.zr22 = -(r22 + r22);
  d.zi11 = -H[0][0] - (i11 + i11);
  d.zi12 = -H[0][1] - (i12 + i21);
  d.zi22 = -H[1][1] - (i22 + i22);
  const double gr = lq.gll_re[l], gi = lq.gll_im[l];
  d.Are = gr * y.Are - gi * y.Aim;
  d.Aim = gr * y.Aim + gi * y.Are;
  d.Lam = lq.lam_rate[l];
}

// One classical RK4 step of size h on component l, into out.
__host__ __device__ inline void rk4_lq(const DevLQ &lq, int l, const OdeLQ &y, double h, OdeLQ &out) {
  OdeLQ ys = y, d;
  const double h6 = h / 6.0;
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    rhs_lq(lq, l, ys, d);
    const double c = st == 2 ? h : 0.5 * h;
    if (st == 0) {
#define F(f) out.f = d.f; ys.f = y.f + c * d.f;
      SHGB_ODELQ_FIELDS(F)
#undef F
    } else if (st < 3) {
#define F(f) out.f = out.f + 2.0 * d.f; ys.f = y.f + c * d.f;
      SHGB_ODELQ_FIELDS(F)
#undef F
    } else {
#define F(f) out.f = y.f + h6 * (out.f + d.f);
      SHGB_ODELQ_FIELDS(F)
#undef F
    }
  }
}

// One call of the interval algorithm (Sec. 2.4 steps 3-5): a trial over the
// rest of the interval, the shortened step to the hop time, or a new trial
// after a hop; true when the interval is complete.  Each lane runs its own
// sequence of calls (see IvPos).
__host__ __device__ inline bool interval_lq_call(const DevLQ &lq, OdeLQ &y, HopScalars &h, IvPos &iv, uint64_t gid,
                                                 uint64_t seed, Counters &cnt) {
  OdeLQ yn;
  rk4_lq(lq, h.comp, y, iv.hstep, yn);
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
  hop_choose_lq(lq, h, gid, seed, cnt);
  ++iv.hops;
  iv.rem = iv.rem * (1.0 - iv.theta);
  if (!(iv.rem > 0.0)) return true;
  iv.hstep = iv.rem;
  return false;
}

__global__ void __launch_bounds__(256)
step_lq_kernel(DevLQ lq, double *__restrict__ tr, double *__restrict__ sc, int32_t *__restrict__ comp,
               uint32_t *__restrict__ nhop, int64_t n, int64_t ld, uint64_t gid0, int nsteps, double dt,
               uint64_t seed, uint64_t *diag) {
  const Layout L(2, ld);
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Counters cnt;
  if (b < n) {
    OdeLQ y;
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
      if (interval_lq_call(lq, y, h, iv, gid, seed, cnt)) {
        ++s;
        iv_begin(iv, dt);
      }
    }
    double chk = h.logw + h.phre + h.phim;
#define F(f) chk += y.f;
    SHGB_ODELQ_FIELDS(F)
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
hop_lq_kernel(DevLQ lq, double *__restrict__ sc, int32_t *__restrict__ comp, uint32_t *__restrict__ nhop, int64_t n,
              int64_t ld, uint64_t gid0, const int32_t *__restrict__ idx, int64_t n_idx, uint64_t seed,
              uint64_t *diag) {
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
      hop_choose_lq(lq, h, gid0 + (uint64_t)b, seed, cnt);
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

hipError_t launch_step_lq(const DevLQ &lq, const shgb_state &st, int nsteps, double dt, uint64_t seed,
                          uint64_t *diag, hipStream_t stream) {
  if (st.n_beams == 0 || nsteps == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (st.n_beams + threads - 1) / threads;
  hipLaunchKernelGGL(step_lq_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, lq, st.f64,
                     scalar_block(st), st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, nsteps, dt, seed,
                     diag);
  return hipGetLastError();
}

hipError_t launch_hop_lq(const DevLQ &lq, const shgb_state &st, const int32_t *idx, int64_t n_idx, uint64_t seed,
                         uint64_t *diag, hipStream_t stream) {
  if (n_idx == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (n_idx + threads - 1) / threads;
  hipLaunchKernelGGL(hop_lq_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, lq, scalar_block(st),
                     st.comp, st.nhop, st.n_beams, st.ld, st.beam_id_offset, idx, n_idx, seed, diag);
  return hipGetLastError();
}

}  // namespace shgb
