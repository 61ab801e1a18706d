// The pair-group layout of a beam with phase space m = 2d > 2 over a group
// of LPB lanes, and the right-hand side of its beam ODEs (Sec. 2.3
// eq:shgb_odes with the arrowhead Hessian of the QCLE with a harmonic bath,
// Sec. 3.3), generic in the element type T of the stage values: float and
// double for the stepping kernels, a (value, derivative) pair for the
// tangent kernel.  The equations and the work split are stated at the top
// of step_wave.hip.
#pragma once

#include "device.h"

namespace shgb {

// Orders the LDS accesses of a beam's lanes, which all sit in one wavefront
// (LPB divides 64): a wavefront executes its LDS accesses in order, so
// wavefront-scope fences (no waits on other memory) and a barrier for the
// compiler suffice.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int D, int LPB>
struct PG {
  static constexpr int M = 2 * D;
  static constexpr int NGRP = D * (D + 1) / 2;          // pair groups a <= b
  static constexpr int NG = (NGRP + LPB - 1) / LPB;     // groups per lane
  static constexpr int G = 64 / LPB;                    // beams per wavefront
  static constexpr int NXP = (M + LPB - 1) / LPB;       // coordinates per lane
  static_assert(64 % LPB == 0, "whole beams per wavefront");
};

// A complex entry of the exchange area: real and imaginary part side by
// side, so that one LDS access moves both.
template <typename T>
struct alignas(2 * sizeof(T)) Cx2 {
  T re, im;
};

// One beam's exchange area (T: the stage precision).  Matrix rows are
// padded to D + 1 entries so that a column read by D lanes does not fall
// into one LDS bank.  sx = sum_{j>0} X_j (bath positions), sp = sum_{j>0}
// P_{d+j}, the two sums the coordinate derivatives need.
template <int D, typename T>
struct PgLds {
  static constexpr int W = D + 1;
  Cx2<T> rp[D][W];   // Zrp
  Cx2<T> pp[D][W];   // Zpp (both triangles)
  Cx2<T> rho[D], chi[D];
  T x[2 * D], p[2 * D];
  T sx, sp;
  T hk[D];           // H_kk = M w_k^2 for k > 0 (hk[0] is not used)
  Cx2<T> xq[D];      // (X_k, P_d+k) side by side, k > 0: the coordinate sums as a row (FP64 stage loop)
};

// Fill the constant part of the exchange area (before the first publish,
// whose barrier orders it before every read).
template <int D, int LPB, typename T>
__device__ inline void pg_fill_const(int r, const double *bath_k, PgLds<D, T> &s) {
  for (int k = r; k < D; k += LPB) s.hk[k] = T(k > 0 ? bath_k[k] : 0.0);
}

// Values of one pair group: Zrr_ab, Zrp_ab, Zrp_ba, Zpp_ab (re, im).
enum { kRrR, kRrI, kAbR, kAbI, kBaR, kBaI, kPpR, kPpI, kGrpN };
template <typename T>
struct Grp {
  T v[kGrpN];
};

// Scalars S and Lam of a beam: FP64 for an FP32 stage, else the stage type.
template <typename T>
struct ScalarOf {
  using type = T;
};
template <>
struct ScalarOf<float> {
  using type = double;
};

// Lane r of the group owns the pair groups r + LPB e and the coordinates
// X_c, P_c, c = r + LPB j.
template <int D, int LPB, typename T>
struct PgY {
  Grp<T> g[PG<D, LPB>::NG];
  T x[PG<D, LPB>::NXP], p[PG<D, LPB>::NXP];
  typename ScalarOf<T>::type S, Lam;
};

template <int D, int LPB, typename T>
struct PgCtx {
  int r;                         // lane within the beam's group
  int a[PG<D, LPB>::NG], b[PG<D, LPB>::NG];  // pair of each owned group, -1: none
};

// The adiabatic quantities along q1 in the stage precision.
template <typename T>
struct Q1T {
  T s, s1, s2, s3, d21;
};

// Write the stage values of the beam's lanes to its exchange area (the
// context may hold another element type than T).
template <int D, int LPB, typename TC, typename T>
__device__ inline void pg_write(const PgCtx<D, LPB, TC> &cx, const PgY<D, LPB, T> &y, PgLds<D, T> &s) {
#pragma unroll
  for (int e = 0; e < PG<D, LPB>::NG; ++e) {
    const int a = cx.a[e], b = cx.b[e];
    if ((e + 1) * LPB <= PG<D, LPB>::NGRP || a >= 0) {   // slots every lane fills need no test
      const T *v = y.g[e].v;
      s.rp[a][b] = Cx2<T>{v[kAbR], v[kAbI]};
      s.rp[b][a] = Cx2<T>{v[kBaR], v[kBaI]};   // a == b: the same entry, written twice with one value
      s.pp[a][b] = Cx2<T>{v[kPpR], v[kPpI]};
      s.pp[b][a] = Cx2<T>{v[kPpR], v[kPpI]};
    }
  }
#pragma unroll
  for (int j = 0; j < PG<D, LPB>::NXP; ++j) {
    const int c = cx.r + LPB * j;
    if (c < 2 * D) { s.x[c] = y.x[j]; s.p[c] = y.p[j]; }
  }
}

// Sum task t < 2D + 1 over k = 1 .. D - 1: t < D: rho_t (row t of Zrp);
// D <= t < 2D: chi_{t-D} (column t - D of Zpp); t = 2D: sx and sp.  The
// operands are picked by address (no branches).
template <int D, typename T>
__device__ inline void pg_sum_task(int t, PgLds<D, T> &s) {
  const bool row = t < D, col = !row && t < 2 * D;
  const int u = row ? t : (col ? t - D : 0);
  const T *br = row ? &s.rp[u][0].re : (col ? &s.pp[0][u].re : &s.x[0]);
  const T *bi = row ? &s.rp[u][0].im : (col ? &s.pp[0][u].im : &s.p[D]);
  const int stride = row ? 2 : (col ? 2 * PgLds<D, T>::W : 1);
  T *orr = row ? &s.rho[u].re : (col ? &s.chi[u].re : &s.sx);
  T *oi = row ? &s.rho[u].im : (col ? &s.chi[u].im : &s.sp);
  T sr = 0, si = 0;
  for (int k = 1; k < D; ++k) { sr += br[k * stride]; si += bi[k * stride]; }
  *orr = sr;
  *oi = si;
}

// The 2D + 1 sums, once the written stage values are visible: one task per
// lane (lanes past the last task repeat it: the same values to the same
// place), round robin when the group has fewer lanes than tasks.
template <int D, int LPB, typename TC, typename T>
__device__ inline void pg_sums(const PgCtx<D, LPB, TC> &cx, PgLds<D, T> &s) {
  if constexpr (2 * D + 1 <= LPB) {
    pg_sum_task<D, T>(cx.r < 2 * D + 1 ? cx.r : 2 * D, s);
  } else {
    for (int t = cx.r; t < 2 * D + 1; t += LPB) pg_sum_task<D, T>(t, s);
  }
}

// Publish the stage values and form the sums rho, chi, sx, sp.
template <int D, int LPB, typename TC, typename T>
__device__ inline void pg_publish(const PgCtx<D, LPB, TC> &cx, const PgY<D, LPB, T> &y, PgLds<D, T> &s) {
  pg_write(cx, y, s);
  wave_lds_sync();
  pg_sums(cx, s);
  wave_lds_sync();
}

// Per-stage scalars of the beam's right-hand side.
template <typename T>
struct StageCoef {
  Q1T<T> k;
  T sg, bc, H00, B00, lam, im;
};

// Derivatives of one pair group (a, b) at the stage values v.
template <int D, typename T>
__device__ inline void grp_deriv(int a, int b, const StageCoef<T> &c, const T *v, const PgLds<D, T> &s, T *d) {
  const T lam = c.lam, im = c.im;
  const T Ha = a == 0 ? c.H00 : s.hk[a], Hb = b == 0 ? c.H00 : s.hk[b];
  // the cross-lane operands, by address select rather than branches
  const Cx2<T> xo = *(b > 0 ? &s.rp[a][0] : &s.rho[a]), to = *(a > 0 ? &s.rp[b][0] : &s.rho[b]);
  const Cx2<T> uo = *(a > 0 ? &s.pp[0][b] : &s.chi[b]), wo = *(b > 0 ? &s.pp[0][a] : &s.chi[a]);
  // Zrr_ab' = (Zrp H)_ab + (Zrp H)_ba
  T xr = v[kAbR] * Hb, xi = v[kAbI] * Hb;
  xr += lam * xo.re;
  xi += lam * xo.im;
  T tr = v[kBaR] * Ha, ti = v[kBaI] * Ha;
  tr += lam * to.re;
  ti += lam * to.im;
  d[kRrR] = xr + tr;
  d[kRrI] = (xi + ti) + ((a == 0 && b == 0) ? c.B00 : (T)0);
  // Zrp_ab' = (H Zpp)_ab - Zrr_ab / M,  Zrp_ba' = (H Zpp)_ba - Zrr_ba / M
  T ur = Ha * v[kPpR], ui = Ha * v[kPpI];
  ur += lam * uo.re;
  ui += lam * uo.im;
  T wr = Hb * v[kPpR], wi = Hb * v[kPpI];
  wr += lam * wo.re;
  wi += lam * wo.im;
  d[kAbR] = ur - v[kRrR] * im;
  d[kAbI] = ui - v[kRrI] * im;
  d[kBaR] = wr - v[kRrR] * im;
  d[kBaI] = wi - v[kRrI] * im;
  // Zpp_ab' = -(Zrp_ba + Zrp_ab) / M
  d[kPpR] = -(v[kBaR] + v[kAbR]) * im;
  d[kPpI] = -(v[kBaI] + v[kAbI]) * im;
}

// Derivatives of the coordinate X_c, P_c (indices c >= m get zeros).  All
// alternatives are formed and one is selected (no branches).
template <int D, typename T>
__device__ inline void xp_deriv(int cc, const StageCoef<T> &c, const PgLds<D, T> &s, T &dx, T &dp) {
  const T lam = c.lam, im = c.im;
  const bool q = cc < D, pm = !q && cc < 2 * D;   // a position, a momentum coordinate
  const int i = q ? cc : (pm ? cc - D : 0);        // the coordinate index
  const T kc = s.hk[i];
  // position: X_i' = p_i / M;  P_i' = d beta / d r_i + (H P_p)_i
  const T dxq = s.x[D + i] * im;
  const T dp0 = c.bc * c.k.s1 + c.H00 * s.p[D] + lam * s.sp;
  const T dpk = kc * s.p[D + i] + lam * s.p[D];
  // momentum: X_{d+i}' = -(grad E)_i;  P_{d+i}' = -P_{r,i} / M
  const T dx0 = -(lam * s.sx + c.sg * c.k.s1);
  const T dxk = -(kc * s.x[i] + lam * s.x[0]);
  const T dpm = -s.p[i] * im;
  const T zero = T(0.0);
  dx = q ? dxq : (pm ? (i == 0 ? dx0 : dxk) : zero);
  dp = q ? (i == 0 ? dp0 : dpk) : (pm ? dpm : zero);
}

}  // namespace shgb
