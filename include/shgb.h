/*
 * shgb.h -- surface hopping Gaussian beam (SHGB) ensemble on AMD Instinct
 * MI355X (gfx950): the C ABI of libshgb.so.
 *
 * Method: Z. Cai and J. Lu, "A surface hopping Gaussian beam method for
 * high-dimensional transport systems", arXiv:1703.06116.  A Monte Carlo
 * ensemble of complex Gaussian beams solves the n-component transport system
 *
 *   d_t u_i + alpha_i(x)^T grad u_i = (i/eps) beta_i(x) u_i + sum_j gamma_ij(x) u_j   (Sec. 1, eq:equations)
 *
 * Each beam follows the characteristic of its current component, carries a
 * phase, a complex Hessian and an amplitude (Sec. 2.3, eq:shgb_odes), hops
 * between components at rates |gamma_jl| (Sec. 2.4) and updates its weight
 * exp(omega).  The solution estimate is U_i(x) = E[exp(omega) G(x) delta_{i,l}]
 * (Sec. 2.3, eq:shgb).
 *
 * The model is the two-level quantum-classical Liouville equation of Sec. 3.3
 * (eq:QCLE and the adiabatic quantities below it) with nuclear mass, as the linear four-component system
 * for (u11, u22, u21, u12 = conj u21); component order 0 = u11 (upper
 * adiabatic surface), 1 = u22 (lower), 2 = u21, 3 = u12.
 *
 * Conventions for every entry point:
 *  - All arrays are device pointers unless stated, owned by the caller.  The
 *    library never allocates or frees device memory; kernels that need scratch
 *    space take a caller workspace whose size a *_workspace query returns.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL is the default
 *    stream) and never synchronise.  Read outputs after synchronising.
 *  - Return 0 (SHGB_OK) or a negative SHGB_E* code; nothing is thrown.
 *    Numerical faults do not fail a call; they are counted in `diag`
 *    (uint64_t[SHGB_NDIAG] on the device, atomically incremented; may be NULL).
 *  - Random numbers: Philox4x64-10 (Salmon et al., SC'11) with key
 *    (seed, 0) and counter (global beam id, draw index, stream tag, 0), so a
 *    beam's draws depend only on its global id and its hop count: sharding
 *    beams or resuming from a saved state never changes them.
 */
#ifndef SHGB_H
#define SHGB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define SHGB_OK 0
#define SHGB_EINVAL (-1)       /* null pointer, bad size, bad parameter     */
#define SHGB_EUNSUPPORTED (-2) /* valid but not built (e.g. model or dimension) */
#define SHGB_EHIP (-3)         /* a HIP launch or runtime call failed        */
#define SHGB_EWORKSPACE (-4)   /* workspace smaller than the query returned  */

/* ---- fixed sizes -------------------------------------------------------- */
#define SHGB_MODEL_QCLE 1
#define SHGB_MODEL_LINQUAD 2
#define SHGB_MODEL_PAPER32 3
#define SHGB_NCOMP 4      /* components (at most, for SHGB_MODEL_LINQUAD)     */
#define SHGB_MAX_D 12     /* nuclear dimensions: phase space m = 2d <= 24     */
#define SHGB_HOP_CAP 16   /* hops per beam per interval; later ones deferred  */

#define SHGB_DIST_NORMAL 0
#define SHGB_DIST_UNIFORM 1

/* diagnostic counters (indices into diag[]) */
#define SHGB_DIAG_HOPS 0          /* hops performed                           */
#define SHGB_DIAG_THR_TIES 1      /* |Lam' - E| <= tau E at a hop test (tau: 1e-12 FP64, 1e-5 MIXED) */
#define SHGB_DIAG_DEST_TIES 2     /* |U R - C_j| <= tau R at a destination draw  */
#define SHGB_DIAG_CAP_OVERFLOW 3  /* intervals that reached SHGB_HOP_CAP hops  */
#define SHGB_DIAG_NONFINITE 4     /* beams with a non-finite state after a call */
#define SHGB_DIAG_NONSPD 5        /* populations: an LDL^T pivot with Re <= 0   */
#define SHGB_DIAG_ZERO_RATE 6     /* hop requested where every rate is zero    */
#define SHGB_DIAG_BAD_INDEX 7     /* shgb_hop: index outside [0, n_beams)      */
#define SHGB_NDIAG 8

/* ---- model -------------------------------------------------------------
 * Two-level QCLE (Sec. 3.3) with nuclear coordinates r = (q1..qd), momenta
 * p = (p1..pd), phase space x = (r, p), m = 2d.  Diabatic potential
 *   V11 =  A tanh(B q1) + Vb(r),  V22 = -A tanh(B q1) + Vb(r),  V12 = C exp(-D q1^2),
 *   Vb(r) = sum_{k=2..d} ( mass w_k^2 q_k^2 / 2 + lam q1 q_k ),
 * adiabatic energies and coupling d21 by the adiabatic energies and d21 below eq:QCLE; transport fields
 * alpha_l = (p/mass, -grad E_l), phases beta = (0, 0, E1-E2, E2-E1), couplings
 * gamma from (p/mass).d21 as in eq:QCLE.  eps is the semiclassical
 * parameter: it enters only the beam shape G, never the beam ODEs.
 *
 * Linear-quadratic systems (the class of Sec. 3.1, eq:ex1 among them):
 * x in R^2 (m = 2, d = 1), n_comp <= SHGB_NCOMP components with
 *   alpha_l(x) = a_l + J_l x,   beta_l(x) = b0_l + b_l.x + x^T H_l x / 2,
 *   gamma_jl constant complex,
 * for which the beam ODEs of Sec. 2.3 are exact (no O(eps^1/2) residual).
 * gamma_ll may be nonzero (then dA/dt = gamma_ll A); a hop from l goes to
 * j != l with probability |gamma_jl| / sum_{k != l} |gamma_kl| and
 * multiplies the phase by gamma_jl / |gamma_jl|.  With x-independent
 * coefficients (a = J = b = H = 0) this is the system of Sec. 2.1.
 * Stepping and hops of this kind are FP64 only.
 *
 * SHGB_MODEL_PAPER32: the two-component system with nonlinear coefficients
 * of Sec. 3.2, eq:ex2, x in R^2 (d = 1), no parameters besides eps:
 *   alpha_1 = -(sin(x1 + x2), cos(x1 - x2)), alpha_2 = -(sin(x1 - x2), cos(x1 + x2)),
 *   beta_1 = sin|x|^2, beta_2 = cos|x|^2, gamma = |x|^2 [[-1, 5], [-5, -1/2]].
 * FP64 stepping and hops.                                                   */
typedef struct shgb_linquad {
  int32_t n_comp;                          /* 1..SHGB_NCOMP                  */
  double a[SHGB_NCOMP][2];
  double J[SHGB_NCOMP][2][2];              /* J_l[i][k] = d alpha_l,i / d x_k */
  double b0[SHGB_NCOMP];
  double b[SHGB_NCOMP][2];
  double H[SHGB_NCOMP][2][2];              /* symmetric                      */
  double gamma_re[SHGB_NCOMP][SHGB_NCOMP]; /* [j][l]: from component l to j  */
  double gamma_im[SHGB_NCOMP][SHGB_NCOMP];
} shgb_linquad;

typedef struct shgb_model {
  int32_t kind;                       /* SHGB_MODEL_QCLE, _LINQUAD or _PAPER32 */
  int32_t d;                          /* 1..SHGB_MAX_D (1 for LINQUAD)      */
  double mass, eps;                   /* > 0 (mass unused by LINQUAD)       */
  double A, B, C, D;                  /* QCLE potential parameters (C != 0) */
  double lam;                         /* QCLE bath coupling (unused when d == 1) */
  double bath_omega[SHGB_MAX_D - 1];  /* QCLE w_2..w_d (> 0), unused when d == 1 */
  shgb_linquad lq;                    /* LINQUAD coefficients (unused by QCLE) */
} shgb_model;

/* ---- beam state --------------------------------------------------------
 * Structure of arrays, beam index fastest: field f of beam b is at
 * [f * ld + b].  With T = m(m+1)/2 the fields are
 *   trajectory rows:  X[m], P[m], Zre[T], Zim[T]          (shgb_traj_fields(m))
 *   scalar rows:      S, Are, Aim, logw, phre, phim, Lam, E (SHGB_SCALAR_FIELDS)
 * Z = M + iN is the complex symmetric beam Hessian (Sec. 2, the beam G^eps) packed
 * by rows of its upper triangle ((i, j), i <= j, at i*m - i(i-1)/2 + j - i);
 * A the complex amplitude; Re omega = logw + Lam where Lam is the rate
 * integral since the last hop; exp(i Im omega) = phre + i phim; E the current
 * waiting-time threshold (the beam hops when Lam reaches E).
 * comp[b] is the current component l_t, nhop[b] the number of hops so far.
 * Beam b has global id beam_id_offset + b.
 *
 * Precision:
 *  - SHGB_FP64: f64 holds the trajectory rows followed by the scalar rows
 *    (shgb_nfields(m) rows); f32 is unused (may be NULL).
 *  - SHGB_MIXED: f32 holds the trajectory rows (shgb_traj_fields(m) rows of
 *    ld floats) and f64 only the scalar rows (SHGB_SCALAR_FIELDS rows).  The
 *    beam ODEs are integrated in FP32; the phase S, the rate integral Lam,
 *    the threshold, the weight and the unit phase stay FP64 (S / eps is a
 *    large angle and Lam decides hop times).  Populations are formed in FP64
 *    from the stored values; the field is evaluated in FP32 with FP64 sums
 *    for m = 2 and as in SHGB_FP64 otherwise.                               */
#define SHGB_FP64 0
#define SHGB_MIXED 1
#define SHGB_SCALAR_FIELDS 8
typedef struct shgb_state {
  double *f64;              /* device: shgb_nfields(m) rows (FP64) or 8 rows (MIXED) of ld */
  int32_t *comp;            /* device, n_beams                      */
  uint32_t *nhop;           /* device, n_beams                      */
  int64_t n_beams;          /* >= 0                                 */
  int64_t ld;               /* >= n_beams                           */
  uint64_t beam_id_offset;
  int32_t m;                /* must equal 2 * model.d               */
  int32_t precision;        /* SHGB_FP64 or SHGB_MIXED              */
  float *f32;               /* device, MIXED: shgb_traj_fields(m) rows of ld */
} shgb_state;

/* trajectory rows per beam for phase-space dimension m */
static inline int32_t shgb_traj_fields(int32_t m) { return 2 * m + m * (m + 1); }
/* double rows per beam of an SHGB_FP64 state */
static inline int32_t shgb_nfields(int32_t m) { return shgb_traj_fields(m) + SHGB_SCALAR_FIELDS; }

/* ---- initial data -------------------------------------------------------
 * Sec. 2.5 and Sec. 2.4 step 2.  Beam shape M0 = I, N0 = 0, P0 = 0, S0 = 0,
 * A0 = a0, or (2 pi eps)^(-m/2) (each beam integrates to one) when a0 == 0,
 * omega = 0, phase 1,
 * all beams on component comp0, a fresh threshold from draw 0.  Centres:
 *   q1 ~ N(q_mean, q_std^2);  p1 ~ N(p_a, p_b^2) or U[p_a, p_b);
 *   bath k >= 2: q_k ~ N(0, eps/(2 mass w_k)), p_k ~ N(0, eps mass w_k / 2)
 * (ground-state Wigner function with hbar -> eps).  Normals by Box-Muller. */
typedef struct shgb_init_spec {
  double q_mean, q_std;
  int32_t p_dist;           /* SHGB_DIST_NORMAL or SHGB_DIST_UNIFORM */
  double p_a, p_b;
  int32_t comp0;            /* 0..n_comp-1 */
  double a0;                /* initial amplitude; 0: (2 pi eps)^(-m/2) */
} shgb_init_spec;

/* Sample every beam of `st` (Sec. 2.5).  Errors: EINVAL for null pointers,
 * m != 2d, ld < n_beams, bad spec. */
int shgb_init_beams(const shgb_model *model, const shgb_init_spec *spec,
                    const shgb_state *st, uint64_t seed, void *stream);

/* Advance every beam by `nsteps` intervals of length dt (Sec. 2.4 steps 3-5):
 * per interval a classical RK4 trial step of the beam ODEs (Sec. 2.3,
 * eq:shgb_odes) on the current component; if the rate integral reaches the
 * threshold, the hop time is found by linear interpolation of Lam, the system
 * is re-integrated to it, the hop is applied (shgb_hop) and the beam finishes
 * the interval on its new component, up to SHGB_HOP_CAP hops per interval.
 * The state is read once and written once per call; nsteps may be large.
 * A SHGB_MIXED state counts threshold ties within 1e-5 E (FP32 trajectories
 * move hop times by about 1e-7 relative).
 * Errors: EINVAL (null pointers, nsteps < 0, dt not finite or <= 0),
 * EUNSUPPORTED (d not built). */
int shgb_step_ensemble(const shgb_model *model, const shgb_state *st, int32_t nsteps,
                       double dt, uint64_t seed, uint64_t *diag, void *stream);

/* shgb_step_ensemble with a choice of Runge-Kutta scheme: SHGB_SCHEME_RK4
 * (classical, as shgb_step_ensemble) or SHGB_SCHEME_RK3 (Kutta's third-order
 * method: Sec. 2.4 integrates the system with a third-order Runge-Kutta
 * method without naming it; k1 = f(y), k2 = f(y + h k1/2),
 * k3 = f(y - h k1 + 2h k2), y + h (k1 + 4 k2 + k3)/6), every trial and
 * shortened step of the interval algorithm taken with it.  RK3: QCLE, d = 1,
 * FP64 state.  Errors: EINVAL (also an unknown scheme), EUNSUPPORTED. */
#define SHGB_SCHEME_RK4 4
#define SHGB_SCHEME_RK3 3
int shgb_step_ensemble_scheme(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt,
                              uint64_t seed, int32_t scheme, uint64_t *diag, void *stream);

/* Apply one hop (Sec. 2.4 step 5) to each listed beam at its current state:
 * destination j != l drawn with probability |gamma_jl| / sum_k |gamma_kl|
 * (inverse CDF over j ascending, uniform U from draw nhop+1), phase times
 * gamma_jl/|gamma_jl|, logw += Lam, Lam = 0, l = j, nhop += 1, new threshold
 * E = -log(1 - Y) from the same draw.  idx: device int32[n_idx], distinct
 * beam indices (duplicates race); indices outside [0, n_beams) are skipped
 * and counted in SHGB_DIAG_BAD_INDEX.  Errors: EINVAL. */
int shgb_hop(const shgb_model *model, const shgb_state *st, const int32_t *idx,
             int64_t n_idx, uint64_t seed, uint64_t *diag, void *stream);

/* Component populations (Sec. 2.3 eq:shgb integrated over x, Sec. 2.4
 * steps 6-7).  Per beam c = exp(logw+Lam) phase A exp(iS/eps)
 * (2 pi eps)^(m/2) det(Z)^(-1/2) exp(-P^T Z^-1 P / (2 eps)) with the branch of
 * det(Z)^(1/2) = prod of principal square roots of the LDL^T pivots.  out:
 * device double[SHGB_NCOMP * 5], per component {sum Re c, sum Im c,
 * sum (Re c)^2, sum (Im c)^2, count}; the population is sum c / N_traj.
 * The reduction order is fixed: results are bitwise reproducible.
 * work: device, >= shgb_populations_workspace(n_beams, m) bytes.
 * Errors: EINVAL, EWORKSPACE. */
int64_t shgb_populations_workspace(int64_t n_beams, int32_t m);
int shgb_populations(const shgb_model *model, const shgb_state *st, double *out,
                     void *work, int64_t work_bytes, uint64_t *diag, void *stream);

/* Sec. 2.4 step 7: the population estimates from the sums of shgb_populations
 * (or of several shards' sums added together) over n_traj >= 1 trajectories.
 * stats: device double[SHGB_NCOMP * 4]; for component i,
 * stats[i*4 + {0, 1}] = Re, Im of the mean sum c / n_traj and
 * stats[i*4 + {2, 3}] = the standard errors of the real and imaginary parts,
 * sqrt((sum x^2 / n_traj - mean^2) / (n_traj - 1)) (variance clipped at zero;
 * n_traj - 1 read as 1 when n_traj == 1).  sums: device double[SHGB_NCOMP * 5].
 * Errors: EINVAL. */
int shgb_population_stats(const double *sums, int64_t n_traj, double *stats, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): shgb_populations
 * with its partial sums in a 320 KiB array that the library holds on each
 * GPU until the process ends, instead of a caller workspace.  Same result,
 * bitwise, as shgb_populations.  The array has room for the partials of any
 * ensemble size (SHGB_EWORKSPACE otherwise); it allocates nothing and every
 * partial is rewritten by each call.  All calls on one GPU share the array:
 * calls that overlap on a GPU (other streams or threads) race and must be
 * serialised by the caller.  Errors: EINVAL, EUNSUPPORTED (m not in
 * {2, 4, 6, 8, 24}), EHIP (the array's device address could not be found). */
int shgb_populations_noalloc(const shgb_model *model, const shgb_state *st, double *out, uint64_t *diag,
                             void *stream);

/* Superposition at Q evaluation points (Sec. 2.3 eq:shgb, Sec. 2.4 step 6):
 * out[(i*Q + q)*2 + {0,1}] = Re, Im of sum_{k: l_k = i} exp(omega_k) G_k(x_q),
 * G(x) = A exp(-(x-X)^T Z (x-X)/(2 eps) + i P.(x-X)/eps + i S/eps), unnormalised
 * (divide by N_traj for U_i).  points: device double[Q * m], row-major.
 * Fixed reduction order (bitwise reproducible for the same beam count and
 * point count: the beam chunks of the sum depend on both).  work: device, >=
 * shgb_reconstruct_workspace(n_beams, m, Q) bytes.  Errors: EINVAL, EWORKSPACE,
 * EUNSUPPORTED (m not in {2, 4, 6, 8, 24}; m = 24 with 2^26 or more beams or
 * points). */
int64_t shgb_reconstruct_workspace(int64_t n_beams, int32_t m, int64_t Q);
int shgb_reconstruct(const shgb_model *model, const shgb_state *st, const double *points,
                     int64_t Q, double *out, void *work, int64_t work_bytes, void *stream);

/* shgb_reconstruct with a choice of arithmetic.  SHGB_FIELD_DEFAULT: as
 * shgb_reconstruct.  SHGB_FIELD_FP32_MATRIX (m = 24): the exponents on the
 * FP32 matrix cores about a centre per tile of 64 beams, the beam weights in
 * FP64, exp and sincos in FP32, FP64 sums.  Its error is stated, not bounded
 * by the FP64 bar: on the 2^18-beam, 2000-interval d = 12 ensemble about
 * 1e-3 of sum_k |exp(omega_k) G_k(x)| at worst and 1e-4 in relative L2
 * norm (squeezed beams lose digits in the quadratic form).  Same workspace
 * rules, queried with shgb_reconstruct_workspace_mode.  Errors: as
 * shgb_reconstruct; EINVAL for an unknown mode, EUNSUPPORTED for the FP32
 * mode with m != 24. */
#define SHGB_FIELD_DEFAULT 0
#define SHGB_FIELD_FP32_MATRIX 1
int64_t shgb_reconstruct_workspace_mode(int64_t n_beams, int32_t m, int64_t Q, int32_t mode);
int shgb_reconstruct_mode(const shgb_model *model, const shgb_state *st, const double *points, int64_t Q,
                          double *out, void *work, int64_t work_bytes, int32_t mode, void *stream);

/* ---- pathwise derivative of the populations ----------------------------
 * The derivative of the population sums (Sec. 2.3 eq:shgb integrated,
 * as shgb_populations) after nsteps intervals, with respect to
 * theta = (A, B, C, D, p_mean): the potential parameters and a common
 * shift of every beam's initial p1 (the mean initial momentum).  The
 * discrete algorithm is differentiated with its events frozen: hop tests,
 * destinations and phase signs are taken at the values exactly as
 * shgb_step_ensemble takes them, the drawn thresholds carry no derivative,
 * and the hop time moves with the parameters through
 * theta = (E - Lam)/(Lam' - Lam) and the shortened step it sets.  This is
 * the limit of central differences with common random numbers while no
 * event flips.  Forward (tangent) propagation, one pass per requested
 * direction; QCLE with d = 1 (m = 2) or with a harmonic bath and
 * d in {2, 3, 4, 12}, FP64 state.  For d > 1, p_mean shifts p1 only.
 *
 * st: the initial ensemble (read, never written).  dir_mask: bit j selects
 * theta_j.  out: device double[5 * SHGB_NCOMP * 4]; for direction j and
 * component i, out[(j * SHGB_NCOMP + i) * 4 + {0, 1, 2, 3}] = sum Re c,
 * sum Im c, d/dtheta_j sum Re c, d/dtheta_j sum Im c over the beams on
 * component i at the end (entries of unselected directions are left as
 * they were).  work: device, >= shgb_population_tangent_workspace(n_beams).
 * Errors: EINVAL, EWORKSPACE, EUNSUPPORTED (other d, mixed state, LINQUAD or
 * eq:ex2 model). */
#define SHGB_NTHETA 5
int64_t shgb_population_tangent_workspace(int64_t n_beams);
int shgb_population_tangent(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt,
                            uint64_t seed, uint32_t dir_mask, double *out, void *work, int64_t work_bytes,
                            uint64_t *diag, void *stream);

/* ---- reverse-mode (adjoint) derivative of the populations ---------------
 * The gradient of a scalar objective of the populations after nsteps
 * intervals (Sec. 2.3 eq:shgb integrated over x, Sec. 2.4 steps 3-7),
 *   L = sum_i (cot[2i] Re U_i + cot[2i+1] Im U_i),
 *   U_i = (1 / n_traj) sum_{l_k = i} c_k   (c_k as in shgb_populations),
 * with respect to theta = (A, B, C, D, p_mean), in one reverse sweep for all
 * five.  The derivative is the one shgb_population_tangent propagates
 * forwards (events frozen at the values, thresholds without derivative,
 * hop times moving through theta = (E - Lam)/(Lam' - Lam)).
 *
 * Use: shgb_step_checkpointed advances the ensemble exactly as
 * shgb_step_ensemble does and writes the whole state before every segment
 * of `every` intervals into ckpt (caller memory of shgb_checkpoint_bytes);
 * shgb_population_adjoint then takes the stepped state, the checkpoints and
 * the same nsteps, dt, seed and every, runs each segment forward again from
 * its checkpoint and sweeps it backwards.  cot: device double[SHGB_NCOMP * 2];
 * out: device double[6] = dL/dA, dL/dB, dL/dC, dL/dD, dL/dp_mean, L.
 * QCLE, FP64 state, d in {1, 2, 3, 4, 12} (the workspace query returns -1
 * for other m).  For d > 1 the beams are taken in chunks of at most 65536;
 * the workspace holds one segment's stage records for a chunk (8 (4 (3 + 4d)
 * + 2) bytes per beam and interval), the chunk's adjoint states and a copy
 * of its checkpoint.  Errors: EINVAL, EWORKSPACE, EUNSUPPORTED. */
int64_t shgb_checkpoint_bytes(int64_t n_beams, int32_t m, int32_t nsteps, int32_t every);
int shgb_step_checkpointed(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt, uint64_t seed,
                           int32_t every, void *ckpt, int64_t ckpt_bytes, uint64_t *diag, void *stream);
int64_t shgb_population_adjoint_workspace(int64_t n_beams, int32_t m, int32_t every);
int shgb_population_adjoint(const shgb_model *model, const shgb_state *st, const void *ckpt, int32_t nsteps, double dt,
                            uint64_t seed, int32_t every, const double *cot, int64_t n_traj, double *out, void *work,
                            int64_t work_bytes, void *stream);

/* ---- the same derivative with the forward run's stage records kept ------
 * Memory instead of recomputation (d in {2, 3, 4, 12}, FP64): the reverse
 * sweep above runs every segment forward a second time to get the stage
 * records its vector-Jacobian products read (Sec. 2.3 eq:shgb_odes through
 * the RK4 stages of Sec. 2.4 step 3).  shgb_step_recorded advances the
 * ensemble as shgb_step_checkpointed does (the same checkpoints, the same
 * final state, hops and diag counts) and also writes those records of every
 * interval into recs, and the start state of each interval with a hop into
 * one of 4 slots per beam and segment (the reverse sweep starts such an
 * interval there instead of running its segment again up to it; a beam's
 * fifth and later hop intervals of a segment get no slot): device memory of
 * shgb_record_bytes, per beam and whole segment of `every` intervals
 * 8 every (4 (3 + 4d) + 2) bytes of records and 4 slots of
 * 8 (2m + m (m + 1) + 5, rounded up to even) bytes (d = 12: 1648 bytes per
 * beam and interval and 4 x 5232 bytes per beam and segment, 122 GB for
 * 65536 beams and 1000 intervals in segments of 100).  Segment c, beam b,
 * interval i of the segment at recs + ((c n_beams + b) every + i)
 * (4 (3 + 4d) + 2) doubles; the slots after the n_seg segments' records.
 * shgb_population_adjoint_recorded then gives what shgb_population_adjoint
 * gives for the same stepped state and checkpoints, without the replays; its
 * workspace (shgb_population_adjoint_recorded_workspace) holds no records.
 * The caller owns ckpt, recs and work; the two calls must see the same
 * nsteps, dt, seed and every, and recs unchanged between them.
 * shgb_record_bytes and the workspace query return -1 for m = 2 and other d.
 * Errors: EINVAL, EWORKSPACE (ckpt or recs too small), EUNSUPPORTED (m = 2,
 * other d, mixed state, other models). */
int64_t shgb_record_bytes(int64_t n_beams, int32_t m, int32_t nsteps, int32_t every);
int shgb_step_recorded(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt, uint64_t seed,
                       int32_t every, void *ckpt, int64_t ckpt_bytes, double *recs, int64_t recs_bytes,
                       uint64_t *diag, void *stream);
int64_t shgb_population_adjoint_recorded_workspace(int64_t n_beams, int32_t m, int32_t every);
int shgb_population_adjoint_recorded(const shgb_model *model, const shgb_state *st, const void *ckpt,
                                     const double *recs, int32_t nsteps, double dt, uint64_t seed, int32_t every,
                                     const double *cot, int64_t n_traj, double *out, void *work, int64_t work_bytes,
                                     void *stream);

/* ---- batches: many instances in one persistent launch ------------------
 * A batch is n_inst independent QCLE instances (model, state, seed) of one
 * dimension d and one precision; models may differ in every parameter and
 * states in size.  Each instance's beams are cut into tiles of one
 * workgroup's worth; a fixed grid of workgroups takes tiles from a device
 * queue until none is left, so uneven instance sizes and hop histories
 * balance across the GPU.  Results are bitwise those of shgb_step_ensemble
 * on each instance alone (the per-beam arithmetic is the same).
 *
 * Use: shgb_batch_prepare writes the instance table into host memory and
 * fills `batch`; the caller copies the table to device memory (it must stay
 * there while the batch is used), sets batch->table to that copy, and calls
 * shgb_step_batched as often as wanted.  The launch sequence of
 * shgb_step_batched (a queue reset kernel and the persistent kernel; no
 * memset, no allocation, no synchronisation) can be captured in a HIP graph.
 * Calls that share a work buffer must not overlap. */
typedef struct shgb_batch_config {
  int32_t waves_per_block;  /* 2 or 4; a tile is 64*w beams (m = 2), 2w (m = 24), 8w (m = 4, 6, 8) */
  int32_t blocks_per_cu;    /* persistent workgroups per compute unit, 1..16 */
  int32_t tiles_per_grab;   /* tiles taken from the queue at once, >= 1 */
} shgb_batch_config;

typedef struct shgb_batch {
  int32_t n_inst, d, precision, kind;
  int64_t total_tiles;
  shgb_batch_config cfg;
  const void *table;        /* device copy of the table (set by the caller) */
} shgb_batch;

#define SHGB_BATCH_WORK_BYTES 256  /* device work buffer of shgb_step_batched */

/* bytes of the host table for n_inst instances (-1 if n_inst < 1) */
int64_t shgb_batch_table_bytes(int32_t n_inst);
/* Validate the instances (each as shgb_step_ensemble would) and write the
 * table.  models, states, seeds: host arrays of n_inst.  Errors: EINVAL
 * (bad instance, mixed d or precision, bad config, table too small),
 * EUNSUPPORTED (a kind or d without a batched kernel). */
int shgb_batch_prepare(const shgb_model *models, const shgb_state *states, const uint64_t *seeds,
                       int32_t n_inst, const shgb_batch_config *cfg, void *host_table,
                       int64_t table_bytes, shgb_batch *batch);
/* Advance every instance of the batch by nsteps intervals of dt (the
 * algorithm of shgb_step_ensemble).  work: device, >= SHGB_BATCH_WORK_BYTES.
 * diag: counters summed over the batch.  Errors: EINVAL. */
int shgb_step_batched(const shgb_batch *batch, int32_t nsteps, double dt, void *work, int64_t work_bytes,
                      uint64_t *diag, void *stream);

/* Diagnostic: the raw Philox4x64-10 blocks for n counters (device
 * uint64[4n] in and out) under key (seed, 0), as the kernels draw them. */
int shgb_philox(uint64_t seed, const uint64_t *counters, uint64_t *out, int64_t n, void *stream);

/* sizeof(shgb_model), sizeof(shgb_state), sizeof(shgb_init_spec),
 * sizeof(shgb_batch_config), sizeof(shgb_batch) into sizes[0..4] (host
 * array), so bindings can check their struct layouts. */
void shgb_abi_sizes(int64_t *sizes);

const char *shgb_strerror(int code);
int32_t shgb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SHGB_H */
