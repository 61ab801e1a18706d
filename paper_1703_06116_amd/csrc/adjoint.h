// Building blocks of the reverse-mode (adjoint) derivative of the
// populations: the Jacobian of the QCLE two-level quantities with respect to
// q1 and the potential parameters, the leg structure of one interval of the
// hop algorithm, and the checkpoint layout shared by the forward entry point
// and the reverse kernels.
//
// The derivative is that of the discrete algorithm with its events frozen
// (the same one the tangent kernels propagate forwards): every hop test,
// destination and phase sign is decided by the values, the drawn thresholds
// carry no derivative, and a hop time moves with the state through
// theta = (E - Lam)/(Lam' - Lam) (Sec. 2.4 step 4) and the shortened step it
// sets.  Adjoint variables of the packed Hessian entries are the partial
// derivatives with respect to the packed (stored) variables.
#pragma once

#include "cplx.h"
#include "device.h"

namespace shgb {

// Adjoints (sb[o], o = s, s1, s2, s3, d21) of the two-level quantities of
// Sec. 3.3 (the adiabatic energies and d21 below eq:QCLE, as qcle_q1 forms
// them) pulled back to q1 (returned) and to (A, B, C, D) (added to th_out),
// by a reverse sweep through the scalar formulas: th = tanh(x) and sech2 = 1 - th^2 with x = B q1 have th' = sech2 and
// sech2' = -2 th sech2; c = C exp(-D q1^2).
__host__ __device__ inline double q1_pullback_rev(const DevModel &md, double q, const double sb[5], double th_out[4]) {
  const double A = md.A, B = md.B, C = md.C, D = md.D;
  // forward values (as qcle_q1 forms them)
  const double x = B * q;
  const double e = exp(-2.0 * fabs(x));
  const double r = 1.0 / (1.0 + e);
  const double th = copysign((1.0 - e) * r, x);
  const double sech2 = 4.0 * e * r * r;
  const double AB = A * B;
  const double a = A * th, a1 = AB * sech2, a2 = -2.0 * AB * B * th * sech2;
  const double u = 1.0 - 3.0 * th * th;
  const double a3 = -2.0 * AB * B * B * sech2 * u;
  const double qq = q * q;
  const double E = exp(-D * qq);
  const double c = C * E;
  const double c1 = -2.0 * D * q * c;
  const double w2 = 4.0 * D * D * qq - 2.0 * D;
  const double c2 = w2 * c;
  const double w3 = 12.0 * D * D - 8.0 * D * D * D * qq;
  const double c3 = q * w3 * c;
  const double ss = a * a + c * c;
  const double rs = 1.0 / sqrt(ss);
  const double N1 = a * a1 + c * c1;
  const double s1 = N1 * rs;
  const double N2 = (a1 * a1 + a * a2) + (c1 * c1 + c * c2) - s1 * s1;
  const double s2 = N2 * rs;
  const double N3 = 3.0 * (a1 * a2 + c1 * c2) + (a * a3 + c * c3) - 3.0 * s1 * s2;
  // reverse sweep
  double ab = 0, a1b = 0, a2b = 0, a3b = 0, cb = 0, c1b = 0, c2b = 0, c3b = 0, rsb = 0, ssb = 0;
  // d21 = (a c1 - c a1) rs^2 / 2
  const double sd = sb[4];
  ab += 0.5 * c1 * rs * rs * sd;
  c1b += 0.5 * a * rs * rs * sd;
  cb -= 0.5 * a1 * rs * rs * sd;
  a1b -= 0.5 * c * rs * rs * sd;
  rsb += (a * c1 - c * a1) * rs * sd;
  // s3 = N3 rs
  const double n3b = sb[3] * rs;
  rsb += N3 * sb[3];
  a1b += 3.0 * a2 * n3b;
  a2b += 3.0 * a1 * n3b;
  c1b += 3.0 * c2 * n3b;
  c2b += 3.0 * c1 * n3b;
  ab += a3 * n3b;
  a3b += a * n3b;
  cb += c3 * n3b;
  c3b += c * n3b;
  const double s2b = sb[2] - 3.0 * s1 * n3b;
  double s1b = sb[1] - 3.0 * s2 * n3b;
  // s2 = N2 rs
  const double n2b = s2b * rs;
  rsb += N2 * s2b;
  a1b += 2.0 * a1 * n2b;
  ab += a2 * n2b;
  a2b += a * n2b;
  c1b += 2.0 * c1 * n2b;
  cb += c2 * n2b;
  c2b += c * n2b;
  s1b -= 2.0 * s1 * n2b;
  // s1 = N1 rs
  const double n1b = s1b * rs;
  rsb += N1 * s1b;
  ab += a1 * n1b;
  a1b += a * n1b;
  cb += c1 * n1b;
  c1b += c * n1b;
  // s = ss rs, rs = ss^(-1/2), ss = a^2 + c^2
  ssb += rs * sb[0];
  rsb += ss * sb[0];
  ssb += -0.5 * rs * rs * rs * rsb;
  ab += 2.0 * a * ssb;
  cb += 2.0 * c * ssb;
  // the tanh chain
  double Ab = th * ab, ABb = sech2 * a1b, Bb = 0.0, thb = A * ab, sechb = AB * a1b;
  ABb += -2.0 * B * th * sech2 * a2b;
  Bb += -2.0 * AB * th * sech2 * a2b;
  thb += -2.0 * AB * B * sech2 * a2b;
  sechb += -2.0 * AB * B * th * a2b;
  ABb += -2.0 * B * B * sech2 * u * a3b;
  Bb += -4.0 * AB * B * sech2 * u * a3b;
  sechb += -2.0 * AB * B * B * u * a3b;
  thb += 12.0 * AB * B * B * sech2 * th * a3b;
  Ab += B * ABb;
  Bb += A * ABb;
  const double xb = thb * sech2 - 2.0 * th * sech2 * sechb;
  double qb = B * xb;
  Bb += q * xb;
  // the Gaussian chain
  double Db = 0.0;
  cb += -2.0 * D * q * c1b;
  Db += -2.0 * q * c * c1b;
  qb += -2.0 * D * c * c1b;
  cb += w2 * c2b;
  Db += (8.0 * D * qq - 2.0) * c * c2b;
  qb += 8.0 * D * D * q * c * c2b;
  cb += q * w3 * c3b;
  qb += (w3 - 16.0 * D * D * D * qq) * c * c3b;
  Db += q * (24.0 * D - 24.0 * D * D * qq) * c * c3b;
  const double Cb = E * cb, Eb = C * cb;
  Db += -qq * E * Eb;
  qb += -2.0 * D * q * E * Eb;
  th_out[0] += Ab;
  th_out[1] += Bb;
  th_out[2] += Cb;
  th_out[3] += Db;
  return qb;
}

// Interval legs (Sec. 2.4 steps 3-5).  An interval is run as legs: a leg
// starts at a state y on component l with rem of the interval left, takes
// the trial step y' = Phi_rem(y), and either ends the interval (no hop:
// y' is the result) or hops at the interpolated time (the shortened step
// Phi_{theta rem}(y), then the weight update logw += Lam, Lam = 0, and the
// next leg with rem (1 - theta) on the new component).
enum LegKind : int { kLegAccept = 0, kLegPartial = 1, kLegEnd = 2, kLegNow = 3 };

// Stage records of the reverse sweep of a d > 1 beam: what the
// vector-Jacobian product of the right-hand side reads of a stage value (the
// centre enters only through q1, p1 and the momentum component of P, the
// Hessian only through dL/dH00 = 2 sum_a G_a0 Z_a,d): per RK4 stage
// q1, p1, P_p1, then Re Zrp_a0, Im Zrp_a0, Re Zpp_0a, Im Zpp_0a for
// a = 0 .. d-1 (one row of d values each); per interval the four stages'
// records, the component and whether the interval has a hop (1.0) or not.
__host__ __device__ constexpr int adj_stage_rec(int d) { return 3 + 4 * d; }
__host__ __device__ constexpr int adj_interval_rec(int d) { return 4 * adj_stage_rec(d) + 2; }

// Start states of the intervals with a hop.  The recording stepping kernel
// writes the state at the start of each interval of a segment on which the
// beam hops into one of kAdjSlots slots of the beam (slot k for the interval
// that starts with k hops made in the segment; later ones get none), and
// the interval's hop flag in its record says which: 0 no hop, k + 1 slot k,
// -1 a hop without a slot.  The reverse sweep starts such an interval from
// its slot instead of running the segment again from its checkpoint up to
// it.  A slot: the trajectory rows (ld = 1), then S, Lam, E, comp, nhop,
// padded to an even count of doubles (16-byte aligned slots).
constexpr int kAdjSlots = 4;
__host__ __device__ constexpr int adj_slot_doubles(int d) {
  return (2 * (2 * d) + (2 * d) * (2 * d + 1) + 5 + 1) / 2 * 2;
}

// Per-block partial sums of the reverse kernels: dA, dB, dC, dD, dp_mean, the
// objective, two unused.
constexpr int kAdjVals = 8;

// ---------------------------------------------------------------------------
// Checkpoints: every `every` intervals the whole state of every beam, in the
// state layout with ld = n (the FP64 rows, then comp and nhop as int32).
struct CkptLayout {
  int64_t n, rows, stride_bytes;  // one checkpoint
  int n_ckpt;
};

__host__ __device__ inline CkptLayout ckpt_layout(int64_t n, int m, int nsteps, int every) {
  CkptLayout c;
  c.n = n;
  c.rows = shgb_nfields(m);
  const int64_t bytes = c.rows * n * 8 + 2 * n * 4;
  c.stride_bytes = (bytes + 255) / 256 * 256;
  c.n_ckpt = (nsteps + every - 1) / every;
  return c;
}

}  // namespace shgb
