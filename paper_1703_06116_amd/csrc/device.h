// Device-side building blocks of libshgb: model parameters, state layout,
// Philox4x64-10, the QCLE coefficient functions and the hop event.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shgb.h"

namespace shgb {

// Kernel-argument copy of the model (by value, no host pointers).
struct DevModel {
  double mass, inv_mass, eps;
  double A, B, C, D, lam;
  // products of the potential parameters used by qcle_q1
  double AB, m2AB2, m2AB3, m2D, D4sq, D12sq, D8cu;
  double bath_w[SHGB_MAX_D];  // w_k for bath modes k = 1..d-1 (index 0 unused)
  double bath_k[SHGB_MAX_D];  // mass * w_k^2
  int d;
  int kind;                   // SHGB_MODEL_QCLE or SHGB_MODEL_LINQUAD
  int n_comp;
};

// Row offsets of the structure-of-arrays state for phase-space dimension m.
// Trajectory rows (X, P, Zre, Zim) live in one block whose element type is
// the state's trajectory precision; the scalar rows live in a double block:
// for an FP64 state that block directly follows the trajectory rows of the
// same array, for a mixed state it is an array of its own.
struct Layout {
  int m, T;
  int64_t ld;
  __host__ __device__ Layout(int m_, int64_t ld_) : m(m_), T(m_ * (m_ + 1) / 2), ld(ld_) {}
  __host__ __device__ int X(int i) const { return i; }
  __host__ __device__ int P(int i) const { return m + i; }
  __host__ __device__ int Zre(int k) const { return 2 * m + k; }
  __host__ __device__ int Zim(int k) const { return 2 * m + T + k; }
  __host__ __device__ int traj_rows() const { return 2 * m + 2 * T; }
  // packed upper-triangle index of (i, j), i <= j
  __host__ __device__ static int tri(int m, int i, int j) { return i * m - i * (i - 1) / 2 + (j - i); }
};

// Rows of the scalar block.
enum ScalarRow : int { kRowS = 0, kRowAre, kRowAim, kRowLogw, kRowPhre, kRowPhim, kRowLam, kRowE };

// Host side: the two blocks of a state.
inline double *scalar_block(const shgb_state &st) {
  return st.precision == SHGB_MIXED ? st.f64 : st.f64 + (int64_t)shgb_traj_fields(st.m) * st.ld;
}
inline bool mixed(const shgb_state &st) { return st.precision == SHGB_MIXED; }

// ---------------------------------------------------------------------------
// Philox4x64-10, from Salmon, Moraes, Dror & Shaw, "Parallel random numbers:
// as easy as 1, 2, 3" (SC'11): ten rounds of two 64x64->128 multiplications
// with the published multipliers, key bumped by the Weyl constants.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

constexpr uint64_t kTagHop = 0x48;     // hop draws: word 0 -> U, word 1 -> Y
constexpr uint64_t kTagNormal = 0x4E;  // Box-Muller normals, 4 per block
constexpr uint64_t kTagUnif = 0x55;    // one uniform per coordinate

struct U64x4 { uint64_t v[4]; };

__host__ __device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  lo = a * b;
  hi = __umul64hi(a, b);
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  lo = (uint64_t)p;
  hi = (uint64_t)(p >> 64);
#endif
}

__host__ __device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += kPhiloxW0; k1 += kPhiloxW1; }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(kPhiloxM0, c0, hi0, lo0);
    mulhilo64(kPhiloxM1, c2, hi1, lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return U64x4{{c0, c1, c2, c3}};
}

__host__ __device__ inline U64x4 draw(uint64_t seed, uint64_t gid, uint64_t index, uint64_t tag) {
  return philox4x64_10(gid, index, tag, 0, seed, 0);
}

// A 64-bit word to a double strictly inside (0, 1): ((w >> 12) + 1/2) 2^-52.
__host__ __device__ inline double u01(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

// ---------------------------------------------------------------------------
// QCLE adiabatic quantities along q1 (Sec. 3.3, the adiabatic energies and d21 below eq:QCLE):
//   a = A tanh(Bq), c = C exp(-Dq^2), s = sqrt(a^2 + c^2) = (E1 - E2)/2,
//   d21 = (a c' - c a') / (2 s^2);
// with derivatives of s up to third order (the Hessian of E feeds the beam
// Jacobian, the third derivative the curvature of P . alpha).
struct Q1 { double s, s1, s2, s3, d21; };

// 1/x from the hardware reciprocal refined by two Newton steps (x > 0, normal).
__host__ __device__ inline double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
#else
  return 1.0 / x;
#endif
}

// 1/sqrt(x) from the hardware estimate refined by two Newton steps (x > 0, normal).
__host__ __device__ inline double rsqrt_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  r = r * fma(-hx * r, r, 1.5);
  r = r * fma(-hx * r, r, 1.5);
  return r;
#else
  return 1.0 / sqrt(x);
#endif
}

__host__ __device__ inline Q1 qcle_q1(const DevModel &md, double q) {
  // tanh and sech^2 from one exponential, accurate in the tails
  const double x = md.B * q;
  const double e = exp(-2.0 * fabs(x));
  const double r = recip(1.0 + e);
  const double th = copysign((1.0 - e) * r, x);
  const double sech2 = 4.0 * e * r * r;
  const double a = md.A * th;
  const double a1 = md.AB * sech2;
  const double a2 = md.m2AB2 * th * sech2;
  const double a3 = md.m2AB3 * sech2 * fma(-3.0 * th, th, 1.0);
  const double q2 = q * q;
  const double c = md.C * exp(-md.D * q2);
  const double c1 = md.m2D * q * c;
  const double c2 = fma(md.D4sq, q2, md.m2D) * c;
  const double c3 = q * fma(-md.D8cu, q2, md.D12sq) * c;
  const double ss = fma(a, a, c * c);
  const double rs = rsqrt_nr(ss);
  Q1 o;
  o.s = ss * rs;
  o.s1 = fma(a, a1, c * c1) * rs;
  o.s2 = (fma(a1, a1, a * a2) + fma(c1, c1, c * c2) - o.s1 * o.s1) * rs;
  o.s3 = (3.0 * fma(a1, a2, c1 * c2) + fma(a, a3, c * c3) - 3.0 * o.s1 * o.s2) * rs;
  o.d21 = 0.5 * fma(a, c1, -c * a1) * rs * rs;
  return o;
}

// The same quantities in FP32 for mixed-precision trajectories: hardware
// exp, reciprocal and reciprocal square root (about 1 ulp each).
struct QcleF {
  float inv_mass, A, B, C, D, lam, AB, m2AB2, m2AB3, m2D, D4sq, D12sq, D8cu;
};

__host__ __device__ inline QcleF qcle_f32(const DevModel &md) {
  QcleF f;
  f.inv_mass = (float)md.inv_mass;
  f.A = (float)md.A;
  f.B = (float)md.B;
  f.C = (float)md.C;
  f.D = (float)md.D;
  f.lam = (float)md.lam;
  f.AB = (float)md.AB;
  f.m2AB2 = (float)md.m2AB2;
  f.m2AB3 = (float)md.m2AB3;
  f.m2D = (float)md.m2D;
  f.D4sq = (float)md.D4sq;
  f.D12sq = (float)md.D12sq;
  f.D8cu = (float)md.D8cu;
  return f;
}

struct Q1f { float s, s1, s2, s3, d21; };

// Host builds (CPU harnesses) use the C library in place of the hardware
// approximations.
__host__ __device__ inline float exp_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __expf(x);
#else
  return expf(x);
#endif
}
__host__ __device__ inline float rcp_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ inline float rsq_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}

__host__ __device__ inline Q1f qcle_q1f(const QcleF &md, float q) {
  const float x = md.B * q;
  const float e = exp_f32(-2.0f * fabsf(x));
  const float r = rcp_f32(1.0f + e);
  const float th = copysignf((1.0f - e) * r, x);
  const float sech2 = 4.0f * e * r * r;
  const float a = md.A * th;
  const float a1 = md.AB * sech2;
  const float a2 = md.m2AB2 * th * sech2;
  const float a3 = md.m2AB3 * sech2 * fmaf(-3.0f * th, th, 1.0f);
  const float q2 = q * q;
  const float c = md.C * exp_f32(-md.D * q2);
  const float c1 = md.m2D * q * c;
  const float c2 = fmaf(md.D4sq, q2, md.m2D) * c;
  const float c3 = q * fmaf(-md.D8cu, q2, md.D12sq) * c;
  const float ss = fmaf(a, a, c * c);
  const float rs = rsq_f32(ss);
  Q1f o;
  o.s = ss * rs;
  o.s1 = fmaf(a, a1, c * c1) * rs;
  o.s2 = (fmaf(a1, a1, a * a2) + fmaf(c1, c1, c * c2) - o.s1 * o.s1) * rs;
  o.s3 = (3.0f * fmaf(a1, a2, c1 * c2) + fmaf(a, a3, c * c3) - 3.0f * o.s1 * o.s2) * rs;
  o.d21 = 0.5f * fmaf(a, c1, -c * a1) * rs * rs;
  return o;
}

// E_l = Vb + sigma_l s and beta_l = bcoef_l s for the four components.
__host__ __device__ inline double comp_sigma(int l) { return l == 0 ? 1.0 : (l == 1 ? -1.0 : 0.0); }
__host__ __device__ inline double comp_bcoef(int l) { return l == 2 ? 2.0 : (l == 3 ? -2.0 : 0.0); }

// Column l of gamma (row j receives from l) for the coupling kappa = (p/M).d21,
// eq:QCLE written for (u11, u22, u21, u12): gamma_jl = sign(l, j) kappa with
//   l = 0: (0, 0, -1, -1);  l = 1: (0, 0, 1, 1);  l = 2, 3: (1, -1, 0, 0).
// Written without branches: hipcc for gfx950 (ROCm 7.2) miscompiled the
// equivalent if/else chain, leaving gamma_1l = 0 for l = 2, 3 in the
// divergent case (the LLVM IR was correct; the machine code lost the store).
__host__ __device__ inline void qcle_gamma_col(int l, double kappa, double col[SHGB_NCOMP]) {
  const double coh = (l >= 2) ? 1.0 : 0.0;                       // leaving u21 or u12
  const double pop = (l == 0) ? -1.0 : ((l == 1) ? 1.0 : 0.0);   // leaving u11 or u22
  col[0] = coh * kappa;
  col[1] = -coh * kappa;
  col[2] = pop * kappa;
  col[3] = pop * kappa;
}

// ---------------------------------------------------------------------------
// Hop event (Sec. 2.4 step 5) on the scalar part of one beam's state.
struct HopScalars {
  double logw, phre, phim, Lam, E;
  int comp;
  uint32_t nhop;
};

struct Counters {
  uint32_t hops = 0, thr_ties = 0, dest_ties = 0, cap = 0, zero_rate = 0, nonfinite = 0;
};

// Where a beam stands inside its current interval [t_n, t_n + dt] of the
// interval algorithm (Sec. 2.4 steps 3-5), for the kernels that run one beam
// per lane with one call per Runge-Kutta step: the time left, the size of the
// next call, the interpolated hop fraction, the hops taken in the interval,
// and whether the next call is the shortened step to a hop time.  Each lane
// runs its own sequence of calls and starts its next interval as soon as it
// completes one, so a wave does not run extra passes for one lane's
// shortened and remaining steps while the others wait.
struct IvPos {
  double rem, hstep, theta;
  int hops;
  bool partial;
};

__host__ __device__ inline void iv_begin(IvPos &iv, double dt) {
  iv.rem = dt;
  iv.hstep = dt;
  iv.theta = 1.0;
  iv.hops = 0;
  iv.partial = false;
}

// Relative bands within which threshold and destination comparisons are
// counted as ties: FP64 trajectories, and FP32 trajectories (mixed states).
constexpr double kTieRel = 1e-12;
constexpr double kTieRelMixed = 1e-5;

// The part of the hop that needs the coupling kappa = (p/M).d21 at the hop
// state: destination, phase jump, component, hop count, next threshold.
// The weight update (logw += Lam, Lam = 0) does not depend on kappa and is
// left to the caller.
__host__ __device__ inline void hop_choose(double kappa, HopScalars &h, uint64_t gid, uint64_t seed, Counters &cnt,
                                           double tie_rel = kTieRel) {
  double col[SHGB_NCOMP];
  qcle_gamma_col(h.comp, kappa, col);
  const U64x4 w = draw(seed, gid, (uint64_t)h.nhop + 1u, kTagHop);
  const double U = u01(w.v[0]);
  const double Y = u01(w.v[1]);
  const int l = h.comp;
  double R = 0.0;
#pragma unroll
  for (int j = 0; j < SHGB_NCOMP; ++j)
    if (j != l) R = R + fabs(col[j]);
  int dest = l;
  if (R > 0.0) {
    const double UR = U * R;
    double C = 0.0;
    int last_pos = l;
    bool chosen = false;
#pragma unroll
    for (int j = 0; j < SHGB_NCOMP; ++j) {
      if (j == l) continue;
      C = C + fabs(col[j]);
      if (fabs(col[j]) > 0.0) last_pos = j;
      if (fabs(UR - C) <= tie_rel * R) cnt.dest_ties++;
      if (!chosen && UR < C) { dest = j; chosen = true; }
    }
    if (!chosen) dest = last_pos;
    if (col[dest] < 0.0) { h.phre = -h.phre; h.phim = -h.phim; }  // gamma/|gamma| = -1
  } else {
    cnt.zero_rate++;
  }
  h.comp = dest;
  h.nhop += 1u;
  h.E = -log(1.0 - Y);
  cnt.hops++;
}

// hop_choose as an out-of-line call, for a loop whose registers are too
// tight to hold the draw inline (the call is made only when a beam hops).
__host__ __device__ __attribute__((noinline)) inline void hop_choose_call(double kappa, HopScalars &h, uint64_t gid,
                                                                          uint64_t seed, Counters &cnt,
                                                                          double tie_rel) {
  hop_choose(kappa, h, gid, seed, cnt, tie_rel);
}

// The whole hop event at phase-space point (q1, p1).
__host__ __device__ inline void hop_event(const DevModel &md, double q1, double p1, HopScalars &h,
                                 uint64_t gid, uint64_t seed, Counters &cnt, double tie_rel = kTieRel) {
  const Q1 k = qcle_q1(md, q1);
  h.logw += h.Lam;
  h.Lam = 0.0;
  hop_choose(p1 * md.inv_mass * k.d21, h, gid, seed, cnt, tie_rel);
}

// ---------------------------------------------------------------------------
// Linear-quadratic model (m = 2) in kernel-argument form.  The constants of
// the hop are formed once on the host: |gamma_jl| with the C library's
// hypot, the unit phase factors gamma_jl / |gamma_jl|, the hop rate
// sum_{j != l} |gamma_jl| summed in ascending j, and the rate integrand
// d Lam / dt = (sum_j |gamma_jl|) - |gamma_ll|.
struct DevLQ {
  int n_comp;
  double a[SHGB_NCOMP][2], J[SHGB_NCOMP][2][2], b0[SHGB_NCOMP], b[SHGB_NCOMP][2], H[SHGB_NCOMP][2][2];
  double gll_re[SHGB_NCOMP], gll_im[SHGB_NCOMP];          // gamma_ll
  double absg[SHGB_NCOMP][SHGB_NCOMP];                     // |gamma_jl|
  double ure[SHGB_NCOMP][SHGB_NCOMP], uim[SHGB_NCOMP][SHGB_NCOMP];  // gamma_jl / |gamma_jl| (0 if gamma_jl = 0)
  double hop_rate[SHGB_NCOMP];                             // sum_{j != l} |gamma_jl|, ascending j
  double lam_rate[SHGB_NCOMP];                             // (sum_j |gamma_jl|) - |gamma_ll|
};

// Hop (Sec. 2.4 step 5) of a linear-quadratic beam: destination by the
// inverse CDF of |gamma_jl| over j != l ascending, phase times
// gamma_jl / |gamma_jl|, then the common updates.
__host__ __device__ inline void hop_choose_lq(const DevLQ &lq, HopScalars &h, uint64_t gid, uint64_t seed,
                                              Counters &cnt, double tie_rel = kTieRel) {
  const U64x4 w = draw(seed, gid, (uint64_t)h.nhop + 1u, kTagHop);
  const double U = u01(w.v[0]);
  const double Y = u01(w.v[1]);
  const int l = h.comp;
  const double R = lq.hop_rate[l];
  int dest = l;
  if (R > 0.0) {
    const double UR = U * R;
    double C = 0.0;
    int last_pos = l;
    bool chosen = false;
    for (int j = 0; j < lq.n_comp; ++j) {
      if (j == l) continue;
      C = C + lq.absg[j][l];
      if (lq.absg[j][l] > 0.0) last_pos = j;
      if (fabs(UR - C) <= tie_rel * R) cnt.dest_ties++;
      if (!chosen && UR < C) { dest = j; chosen = true; }
    }
    if (!chosen) dest = last_pos;
    const double ur = lq.ure[dest][l], ui = lq.uim[dest][l];
    const double pr = h.phre, pi = h.phim;
    h.phre = pr * ur - pi * ui;
    h.phim = pr * ui + pi * ur;
  } else {
    cnt.zero_rate++;
  }
  h.comp = dest;
  h.nhop += 1u;
  h.E = -log(1.0 - Y);
  cnt.hops++;
}

// Hop state of one beam inside a stepping call.  A stepping loop starts a
// hop where the threshold is reached (the weight update, which needs no
// coupling) and completes it (hop_choose) where the coupling at the same
// state is next evaluated: stage 0 of the following RK4 step.
struct HopCtx {
  HopScalars h;
  bool pending;
  uint64_t gid, seed;
};

__host__ __device__ inline void hop_start(HopCtx &hc, double &Lam) {
  hc.h.logw += Lam;
  Lam = 0.0;
  hc.h.Lam = 0.0;
  hc.pending = true;
}

// Wave-level sum of per-lane counters, one atomic per wave and counter.
__device__ inline void flush_counters(const Counters &c, uint64_t *diag) {
  if (!diag) return;
  uint32_t v[6] = {c.hops, c.thr_ties, c.dest_ties, c.cap, c.zero_rate, c.nonfinite};
  const int idx[6] = {SHGB_DIAG_HOPS, SHGB_DIAG_THR_TIES, SHGB_DIAG_DEST_TIES,
                      SHGB_DIAG_CAP_OVERFLOW, SHGB_DIAG_ZERO_RATE, SHGB_DIAG_NONFINITE};
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    uint32_t x = v[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd((unsigned long long *)&diag[idx[t]], (unsigned long long)x);
  }
}

}  // namespace shgb
