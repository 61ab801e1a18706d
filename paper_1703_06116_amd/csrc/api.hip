// The C ABI of libshgb: argument validation, model conversion and dispatch
// to the kernels on the caller's stream.  No device allocation, no
// synchronisation, no exceptions across the boundary.
#include <cmath>
#include <cstring>

#include "adjoint.h"
#include "batch.h"

namespace shgb {
hipError_t launch_init(const DevModel &, const shgb_init_spec &, const shgb_state &, uint64_t, double, hipStream_t);
hipError_t launch_step_lq(const DevLQ &, const shgb_state &, int, double, uint64_t, uint64_t *, hipStream_t);
hipError_t launch_step_p32(const shgb_state &, int, double, uint64_t, uint64_t *, hipStream_t);
hipError_t launch_hop_p32(const shgb_state &, const int32_t *, int64_t, uint64_t, uint64_t *, hipStream_t);
hipError_t launch_hop_lq(const DevLQ &, const shgb_state &, const int32_t *, int64_t, uint64_t, uint64_t *,
                         hipStream_t);
hipError_t launch_step_m2(const DevModel &, const shgb_state &, int, double, uint64_t, uint64_t *, hipStream_t);
hipError_t launch_step_m2_rk3(const DevModel &, const shgb_state &, int, double, uint64_t, uint64_t *, hipStream_t);
hipError_t launch_step_wave(const DevModel &, const shgb_state &, int, double, uint64_t, uint64_t *, hipStream_t);
bool step_wave_supported(int d);
hipError_t launch_hop(const DevModel &, const shgb_state &, const int32_t *, int64_t, uint64_t, uint64_t *,
                      hipStream_t);
hipError_t launch_philox(uint64_t, const uint64_t *, uint64_t *, int64_t, hipStream_t);
int64_t pop_workspace_bytes(int64_t, int);
hipError_t launch_populations(const DevModel &, const shgb_state &, double *, void *, uint64_t *, hipStream_t);
int64_t pop_scratch_bytes();
hipError_t launch_population_stats(const double *, int64_t, double *, hipStream_t);
hipError_t pop_scratch_ptr(void **);
int64_t recon_m2_workspace_bytes(int64_t, int64_t);
hipError_t launch_recon_m2(const DevModel &, const shgb_state &, const double *, int64_t, double *, void *,
                           hipStream_t);
int64_t recon_wave_workspace_bytes(int64_t, int, int64_t);
bool recon_wave_supported(int m);
hipError_t launch_recon_wave(const DevModel &, const shgb_state &, const double *, int64_t, double *, void *,
                             hipStream_t);
int64_t recon_mfma_workspace_bytes(int64_t, int64_t);
bool recon_mfma_supported(int64_t, int64_t);
int wave_tile_beams(int d, int wpb);
int64_t tangent_workspace_bytes(int64_t n);
int64_t tangent_wave_workspace_bytes(int64_t n);
bool tangent_wave_supported(int d);
hipError_t launch_tangent_wave(const DevModel &, const shgb_state &, int, double, uint64_t, uint32_t, double *, void *,
                               uint64_t *, hipStream_t);
hipError_t launch_tangent_m2(const DevModel &, const shgb_state &, int, double, uint64_t, uint32_t, double *, void *,
                             uint64_t *, hipStream_t);
int m2_tile_beams(int wpb);
hipError_t launch_step_checkpointed(const DevModel &, const shgb_state &, int, double, uint64_t, int, void *, double *,
                                    uint64_t *, hipStream_t);
int64_t adj_m2_workspace_bytes(int64_t, int);
int64_t adj_wave_workspace_bytes(int64_t, int, int, bool);
bool adjoint_wave_supported(int d);
hipError_t launch_adjoint_wave(const DevModel &, const shgb_state &, const void *, const double *, int, double,
                               uint64_t, int, const double *, int64_t, double *, void *, hipStream_t);
hipError_t launch_adjoint_m2(const DevModel &, const shgb_state &, const void *, int, double, uint64_t, int,
                             const double *, int64_t, double *, void *, hipStream_t);
hipError_t launch_step_wave_batched(int d, bool mixed_state, int wpb, const BatchItem *items, int n_items,
                                    int64_t total_tiles, int grab, int blocks, int nsteps, double dt,
                                    unsigned long long *queue, uint64_t *diag, hipStream_t stream);
hipError_t launch_step_m2_batched(bool mixed_state, int wpb, const BatchItem *items, int n_items, int64_t total_tiles,
                                  int grab, int blocks, int nsteps, double dt, unsigned long long *queue,
                                  uint64_t *diag, hipStream_t stream);

// Empty the work queue of a batched launch (a kernel, so that graph capture
// records no memset).
__global__ void batch_reset_kernel(unsigned long long *queue) { queue[0] = 0ull; }
hipError_t launch_recon_mfma(const DevModel &, const shgb_state &, const double *, int64_t, double *, void *,
                             hipStream_t);
int64_t recon_mfma32_workspace_bytes(int64_t, int64_t);
bool recon_mfma32_supported(int64_t, int64_t);
hipError_t launch_recon_mfma32(const DevModel &, const shgb_state &, const double *, int64_t, double *, void *,
                               hipStream_t);
}  // namespace shgb

using namespace shgb;

namespace {

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

bool all_finite(const double *v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Linear-quadratic coefficients with the host-side hop constants.
int to_dev_lq(const shgb_linquad &q, DevLQ &lq) {
  if (q.n_comp < 1 || q.n_comp > SHGB_NCOMP) return SHGB_EINVAL;
  std::memset(&lq, 0, sizeof(lq));
  lq.n_comp = q.n_comp;
  const int n = q.n_comp;
  for (int l = 0; l < n; ++l) {
    if (!all_finite(q.a[l], 2) || !all_finite(&q.J[l][0][0], 4) || !std::isfinite(q.b0[l]) ||
        !all_finite(q.b[l], 2) || !all_finite(&q.H[l][0][0], 4) || q.H[l][0][1] != q.H[l][1][0])
      return SHGB_EINVAL;
    std::memcpy(lq.a[l], q.a[l], sizeof(lq.a[l]));
    std::memcpy(lq.J[l], q.J[l], sizeof(lq.J[l]));
    lq.b0[l] = q.b0[l];
    std::memcpy(lq.b[l], q.b[l], sizeof(lq.b[l]));
    std::memcpy(lq.H[l], q.H[l], sizeof(lq.H[l]));
    for (int j = 0; j < n; ++j) {
      const double gr = q.gamma_re[j][l], gi = q.gamma_im[j][l];
      if (!std::isfinite(gr) || !std::isfinite(gi)) return SHGB_EINVAL;
      const double r = std::hypot(gr, gi);
      lq.absg[j][l] = r;
      lq.ure[j][l] = r > 0.0 ? gr / r : 0.0;
      lq.uim[j][l] = r > 0.0 ? gi / r : 0.0;
    }
    lq.gll_re[l] = q.gamma_re[l][l];
    lq.gll_im[l] = q.gamma_im[l][l];
    double R = 0.0, all = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j != l) R = R + lq.absg[j][l];
      all = all + lq.absg[j][l];
    }
    lq.hop_rate[l] = R;
    lq.lam_rate[l] = all - lq.absg[l][l];
  }
  return SHGB_OK;
}

int to_dev_model(const shgb_model *m, DevModel &md, DevLQ *lq = nullptr) {
  if (!m) return SHGB_EINVAL;
  if (m->kind == SHGB_MODEL_PAPER32) {
    if (m->d != 1 || !finite_pos(m->eps)) return SHGB_EINVAL;
    std::memset(&md, 0, sizeof(md));
    md.kind = SHGB_MODEL_PAPER32;
    md.n_comp = 2;
    md.mass = 1.0;
    md.inv_mass = 1.0;
    md.eps = m->eps;
    md.d = 1;
    return SHGB_OK;
  }
  if (m->kind == SHGB_MODEL_LINQUAD) {
    if (m->d != 1 || !finite_pos(m->eps)) return SHGB_EINVAL;
    std::memset(&md, 0, sizeof(md));
    md.kind = SHGB_MODEL_LINQUAD;
    md.n_comp = m->lq.n_comp;
    md.mass = 1.0;
    md.inv_mass = 1.0;
    md.eps = m->eps;
    md.d = 1;
    DevLQ tmp;
    const int rc = to_dev_lq(m->lq, tmp);
    if (rc) return rc;
    if (lq) *lq = tmp;
    return SHGB_OK;
  }
  if (m->kind != SHGB_MODEL_QCLE) return SHGB_EUNSUPPORTED;
  if (m->d < 1 || m->d > SHGB_MAX_D) return SHGB_EINVAL;
  if (!finite_pos(m->mass) || !finite_pos(m->eps)) return SHGB_EINVAL;
  if (!std::isfinite(m->A) || !std::isfinite(m->B) || !std::isfinite(m->C) || !std::isfinite(m->D) ||
      !std::isfinite(m->lam) || m->C == 0.0)
    return SHGB_EINVAL;
  std::memset(&md, 0, sizeof(md));
  md.kind = SHGB_MODEL_QCLE;
  md.n_comp = SHGB_NCOMP;
  md.mass = m->mass;
  md.inv_mass = 1.0 / m->mass;
  md.eps = m->eps;
  md.A = m->A;
  md.B = m->B;
  md.C = m->C;
  md.D = m->D;
  md.lam = m->lam;
  md.AB = m->A * m->B;
  md.m2AB2 = -2.0 * m->A * m->B * m->B;
  md.m2AB3 = -2.0 * m->A * m->B * m->B * m->B;
  md.m2D = -2.0 * m->D;
  md.D4sq = 4.0 * m->D * m->D;
  md.D12sq = 12.0 * m->D * m->D;
  md.D8cu = 8.0 * m->D * m->D * m->D;
  md.d = m->d;
  for (int k = 1; k < m->d; ++k) {
    const double w = m->bath_omega[k - 1];
    if (!finite_pos(w)) return SHGB_EINVAL;
    md.bath_w[k] = w;
    md.bath_k[k] = m->mass * w * w;
  }
  return SHGB_OK;
}

int check_state(const shgb_state *st, const DevModel &md) {
  if (!st) return SHGB_EINVAL;
  if (st->m != 2 * md.d || st->n_beams < 0 || st->ld < st->n_beams) return SHGB_EINVAL;
  if (st->precision != SHGB_FP64 && st->precision != SHGB_MIXED) return SHGB_EINVAL;
  if (st->n_beams > 0 && (!st->f64 || !st->comp || !st->nhop)) return SHGB_EINVAL;
  if (st->n_beams > 0 && st->precision == SHGB_MIXED && !st->f32) return SHGB_EINVAL;
  if (st->n_beams > (int64_t)INT32_MAX) return SHGB_EINVAL;  // beam indices are int32 in shgb_hop
  return SHGB_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? SHGB_OK : SHGB_EHIP; }

}  // namespace

extern "C" {

int shgb_init_beams(const shgb_model *model, const shgb_init_spec *spec, const shgb_state *st, uint64_t seed,
                    void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (!spec) return SHGB_EINVAL;
  if (!std::isfinite(spec->q_mean) || !(spec->q_std >= 0.0) || !std::isfinite(spec->p_a) ||
      !std::isfinite(spec->p_b) || spec->comp0 < 0 || spec->comp0 >= md.n_comp || !std::isfinite(spec->a0))
    return SHGB_EINVAL;
  if (spec->p_dist != SHGB_DIST_NORMAL && spec->p_dist != SHGB_DIST_UNIFORM) return SHGB_EINVAL;
  const double A0 = spec->a0 != 0.0 ? spec->a0 : std::pow(2.0 * M_PI * md.eps, -0.5 * st->m);
  return hip_status(launch_init(md, *spec, *st, seed, A0, (hipStream_t)stream));
}

int shgb_step_ensemble(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt, uint64_t seed,
                       uint64_t *diag, void *stream) {
  DevModel md;
  DevLQ lq;
  int rc = to_dev_model(model, md, &lq);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (nsteps < 0 || !finite_pos(dt)) return SHGB_EINVAL;
  if (md.kind == SHGB_MODEL_LINQUAD) {
    if (st->precision != SHGB_FP64) return SHGB_EUNSUPPORTED;
    return hip_status(launch_step_lq(lq, *st, nsteps, dt, seed, diag, (hipStream_t)stream));
  }
  if (md.kind == SHGB_MODEL_PAPER32) {
    if (st->precision != SHGB_FP64) return SHGB_EUNSUPPORTED;
    return hip_status(launch_step_p32(*st, nsteps, dt, seed, diag, (hipStream_t)stream));
  }
  if (md.d == 1) return hip_status(launch_step_m2(md, *st, nsteps, dt, seed, diag, (hipStream_t)stream));
  if (!step_wave_supported(md.d)) return SHGB_EUNSUPPORTED;
  return hip_status(launch_step_wave(md, *st, nsteps, dt, seed, diag, (hipStream_t)stream));
}

int shgb_step_ensemble_scheme(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt,
                              uint64_t seed, int32_t scheme, uint64_t *diag, void *stream) {
  if (scheme == SHGB_SCHEME_RK4) return shgb_step_ensemble(model, st, nsteps, dt, seed, diag, stream);
  if (scheme != SHGB_SCHEME_RK3) return SHGB_EINVAL;
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (nsteps < 0 || !finite_pos(dt)) return SHGB_EINVAL;
  if (md.kind != SHGB_MODEL_QCLE || md.d != 1 || st->precision != SHGB_FP64) return SHGB_EUNSUPPORTED;
  return hip_status(launch_step_m2_rk3(md, *st, nsteps, dt, seed, diag, (hipStream_t)stream));
}

int shgb_hop(const shgb_model *model, const shgb_state *st, const int32_t *idx, int64_t n_idx, uint64_t seed,
             uint64_t *diag, void *stream) {
  DevModel md;
  DevLQ lq;
  int rc = to_dev_model(model, md, &lq);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (n_idx < 0 || (n_idx > 0 && !idx)) return SHGB_EINVAL;
  if (md.kind == SHGB_MODEL_LINQUAD) {
    if (st->precision != SHGB_FP64) return SHGB_EUNSUPPORTED;
    return hip_status(launch_hop_lq(lq, *st, idx, n_idx, seed, diag, (hipStream_t)stream));
  }
  if (md.kind == SHGB_MODEL_PAPER32) {
    if (st->precision != SHGB_FP64) return SHGB_EUNSUPPORTED;
    return hip_status(launch_hop_p32(*st, idx, n_idx, seed, diag, (hipStream_t)stream));
  }
  return hip_status(launch_hop(md, *st, idx, n_idx, seed, diag, (hipStream_t)stream));
}

int64_t shgb_populations_workspace(int64_t n_beams, int32_t m) {
  if (n_beams < 0 || m < 2 || m > 2 * SHGB_MAX_D || (m & 1)) return -1;
  return pop_workspace_bytes(n_beams, m);
}

int shgb_populations(const shgb_model *model, const shgb_state *st, double *out, void *work, int64_t work_bytes,
                     uint64_t *diag, void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (!out || !work) return SHGB_EINVAL;
  if (st->m != 2 && st->m != 4 && st->m != 6 && st->m != 8 && st->m != 24) return SHGB_EUNSUPPORTED;
  if (work_bytes < pop_workspace_bytes(st->n_beams, st->m)) return SHGB_EWORKSPACE;
  return hip_status(launch_populations(md, *st, out, work, diag, (hipStream_t)stream));
}

int shgb_populations_noalloc(const shgb_model *model, const shgb_state *st, double *out, uint64_t *diag,
                             void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (!out) return SHGB_EINVAL;
  if (st->m != 2 && st->m != 4 && st->m != 6 && st->m != 8 && st->m != 24) return SHGB_EUNSUPPORTED;
  if (pop_workspace_bytes(st->n_beams, st->m) > pop_scratch_bytes()) return SHGB_EWORKSPACE;
  void *work = nullptr;
  if (pop_scratch_ptr(&work) != hipSuccess) return SHGB_EHIP;
  return hip_status(launch_populations(md, *st, out, work, diag, (hipStream_t)stream));
}

int shgb_population_stats(const double *sums, int64_t n_traj, double *stats, void *stream) {
  if (!sums || !stats || n_traj < 1) return SHGB_EINVAL;
  return hip_status(launch_population_stats(sums, n_traj, stats, (hipStream_t)stream));
}

int64_t shgb_reconstruct_workspace(int64_t n_beams, int32_t m, int64_t Q) {
  if (n_beams < 0 || Q < 0 || m < 2 || m > 2 * SHGB_MAX_D || (m & 1)) return -1;
  if (m == 2) return recon_m2_workspace_bytes(n_beams, Q);
  if (m == 24) return recon_mfma_workspace_bytes(n_beams, Q);
  return recon_wave_workspace_bytes(n_beams, m, Q);
}

int shgb_reconstruct(const shgb_model *model, const shgb_state *st, const double *points, int64_t Q, double *out,
                     void *work, int64_t work_bytes, void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (Q < 0 || (Q > 0 && (!points || !out || !work))) return SHGB_EINVAL;
  if (Q > (int64_t)INT32_MAX) return SHGB_EINVAL;
  if (st->m == 2) {
    if (work_bytes < recon_m2_workspace_bytes(st->n_beams, Q)) return SHGB_EWORKSPACE;
    return hip_status(launch_recon_m2(md, *st, points, Q, out, work, (hipStream_t)stream));
  }
  if (st->m == 24) {
    if (!recon_mfma_supported(st->n_beams, Q)) return SHGB_EUNSUPPORTED;
    if (work_bytes < recon_mfma_workspace_bytes(st->n_beams, Q)) return SHGB_EWORKSPACE;
    return hip_status(launch_recon_mfma(md, *st, points, Q, out, work, (hipStream_t)stream));
  }
  if (!recon_wave_supported(st->m)) return SHGB_EUNSUPPORTED;
  if (work_bytes < recon_wave_workspace_bytes(st->n_beams, st->m, Q)) return SHGB_EWORKSPACE;
  return hip_status(launch_recon_wave(md, *st, points, Q, out, work, (hipStream_t)stream));
}

int64_t shgb_reconstruct_workspace_mode(int64_t n_beams, int32_t m, int64_t Q, int32_t mode) {
  if (mode == SHGB_FIELD_DEFAULT) return shgb_reconstruct_workspace(n_beams, m, Q);
  if (mode != SHGB_FIELD_FP32_MATRIX || m != 24 || n_beams < 0 || Q < 0) return -1;
  return recon_mfma32_workspace_bytes(n_beams, Q);
}

int shgb_reconstruct_mode(const shgb_model *model, const shgb_state *st, const double *points, int64_t Q, double *out,
                          void *work, int64_t work_bytes, int32_t mode, void *stream) {
  if (mode == SHGB_FIELD_DEFAULT) return shgb_reconstruct(model, st, points, Q, out, work, work_bytes, stream);
  if (mode != SHGB_FIELD_FP32_MATRIX) return SHGB_EINVAL;
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (Q < 0 || (Q > 0 && (!points || !out || !work))) return SHGB_EINVAL;
  if (Q > (int64_t)INT32_MAX) return SHGB_EINVAL;
  if (st->m != 24 || !recon_mfma32_supported(st->n_beams, Q)) return SHGB_EUNSUPPORTED;
  if (work_bytes < recon_mfma32_workspace_bytes(st->n_beams, Q)) return SHGB_EWORKSPACE;
  return hip_status(launch_recon_mfma32(md, *st, points, Q, out, work, (hipStream_t)stream));
}

// enough for either tangent form (the query does not know m)
static int64_t tangent_work(int64_t n) {
  const int64_t a = tangent_workspace_bytes(n), b = tangent_wave_workspace_bytes(n);
  return a > b ? a : b;
}

int64_t shgb_population_tangent_workspace(int64_t n_beams) {
  if (n_beams < 0) return -1;
  return tangent_work(n_beams);
}

int shgb_population_tangent(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt, uint64_t seed,
                            uint32_t dir_mask, double *out, void *work, int64_t work_bytes, uint64_t *diag,
                            void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (md.kind != SHGB_MODEL_QCLE || st->precision != SHGB_FP64) return SHGB_EUNSUPPORTED;
  if (md.d != 1 && !tangent_wave_supported(md.d)) return SHGB_EUNSUPPORTED;
  if (nsteps < 0 || !finite_pos(dt) || (dir_mask & ~0x1Fu) || !out) return SHGB_EINVAL;
  if (!work || work_bytes < tangent_work(st->n_beams)) return SHGB_EWORKSPACE;
  if (dir_mask == 0) return SHGB_OK;
  if (md.d == 1)
    return hip_status(launch_tangent_m2(md, *st, nsteps, dt, seed, dir_mask, out, work, diag, (hipStream_t)stream));
  return hip_status(launch_tangent_wave(md, *st, nsteps, dt, seed, dir_mask, out, work, diag, (hipStream_t)stream));
}

static bool adjoint_supported(const DevModel &md, const shgb_state *st) {
  return md.kind == SHGB_MODEL_QCLE && st->precision == SHGB_FP64 && (md.d == 1 || adjoint_wave_supported(md.d));
}

int64_t shgb_checkpoint_bytes(int64_t n_beams, int32_t m, int32_t nsteps, int32_t every) {
  if (n_beams < 0 || m < 2 || m > 2 * SHGB_MAX_D || (m & 1) || nsteps < 0 || every < 1) return -1;
  const CkptLayout cl = ckpt_layout(n_beams, m, nsteps, every);
  return (int64_t)cl.n_ckpt * cl.stride_bytes;
}

int shgb_step_checkpointed(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt, uint64_t seed,
                           int32_t every, void *ckpt, int64_t ckpt_bytes, uint64_t *diag, void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (nsteps < 0 || !finite_pos(dt) || every < 1) return SHGB_EINVAL;
  if (!adjoint_supported(md, st)) return SHGB_EUNSUPPORTED;
  const int64_t need = shgb_checkpoint_bytes(st->n_beams, st->m, nsteps, every);
  if (need > 0 && (!ckpt || ckpt_bytes < need)) return SHGB_EWORKSPACE;
  return hip_status(
      launch_step_checkpointed(md, *st, nsteps, dt, seed, every, ckpt, nullptr, diag, (hipStream_t)stream));
}

int64_t shgb_population_adjoint_workspace(int64_t n_beams, int32_t m, int32_t every) {
  if (n_beams < 0 || m < 2 || m > 2 * SHGB_MAX_D || (m & 1) || every < 1) return -1;
  if (m != 2 && !adjoint_wave_supported(m / 2)) return -1;
  return m == 2 ? adj_m2_workspace_bytes(n_beams, every) : adj_wave_workspace_bytes(n_beams, m, every, false);
}

int64_t shgb_record_bytes(int64_t n_beams, int32_t m, int32_t nsteps, int32_t every) {
  if (n_beams < 0 || m < 4 || m > 2 * SHGB_MAX_D || (m & 1) || nsteps < 0 || every < 1) return -1;
  if (!adjoint_wave_supported(m / 2)) return -1;
  const int64_t n_seg = ((int64_t)nsteps + every - 1) / every;
  return n_seg * n_beams * ((int64_t)every * adj_interval_rec(m / 2) + (int64_t)kAdjSlots * adj_slot_doubles(m / 2)) *
         8;
}

int shgb_step_recorded(const shgb_model *model, const shgb_state *st, int32_t nsteps, double dt, uint64_t seed,
                       int32_t every, void *ckpt, int64_t ckpt_bytes, double *recs, int64_t recs_bytes,
                       uint64_t *diag, void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (nsteps < 0 || !finite_pos(dt) || every < 1) return SHGB_EINVAL;
  if (!adjoint_supported(md, st) || st->m == 2) return SHGB_EUNSUPPORTED;
  const int64_t need = shgb_checkpoint_bytes(st->n_beams, st->m, nsteps, every);
  if (need > 0 && (!ckpt || ckpt_bytes < need)) return SHGB_EWORKSPACE;
  const int64_t rneed = shgb_record_bytes(st->n_beams, st->m, nsteps, every);
  if (rneed > 0 && (!recs || recs_bytes < rneed)) return SHGB_EWORKSPACE;
  if (rneed == 0) recs = nullptr;   // nothing to record: the plain kernels
  return hip_status(launch_step_checkpointed(md, *st, nsteps, dt, seed, every, ckpt, recs, diag, (hipStream_t)stream));
}

int64_t shgb_population_adjoint_recorded_workspace(int64_t n_beams, int32_t m, int32_t every) {
  if (n_beams < 0 || m < 4 || m > 2 * SHGB_MAX_D || (m & 1) || every < 1) return -1;
  if (!adjoint_wave_supported(m / 2)) return -1;
  return adj_wave_workspace_bytes(n_beams, m, every, true);
}

int shgb_population_adjoint_recorded(const shgb_model *model, const shgb_state *st, const void *ckpt,
                                     const double *recs, int32_t nsteps, double dt, uint64_t seed, int32_t every,
                                     const double *cot, int64_t n_traj, double *out, void *work, int64_t work_bytes,
                                     void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (nsteps < 0 || !finite_pos(dt) || every < 1 || n_traj < 1 || !cot || !out) return SHGB_EINVAL;
  if (!adjoint_supported(md, st) || st->m == 2) return SHGB_EUNSUPPORTED;
  if (shgb_checkpoint_bytes(st->n_beams, st->m, nsteps, every) > 0 && !ckpt) return SHGB_EINVAL;
  if (shgb_record_bytes(st->n_beams, st->m, nsteps, every) > 0 && !recs) return SHGB_EINVAL;
  if (!work || work_bytes < shgb_population_adjoint_recorded_workspace(st->n_beams, st->m, every))
    return SHGB_EWORKSPACE;
  return hip_status(launch_adjoint_wave(md, *st, ckpt, recs, nsteps, dt, seed, every, cot, n_traj, out, work,
                                        (hipStream_t)stream));
}

int shgb_population_adjoint(const shgb_model *model, const shgb_state *st, const void *ckpt, int32_t nsteps, double dt,
                            uint64_t seed, int32_t every, const double *cot, int64_t n_traj, double *out, void *work,
                            int64_t work_bytes, void *stream) {
  DevModel md;
  int rc = to_dev_model(model, md);
  if (rc) return rc;
  if ((rc = check_state(st, md))) return rc;
  if (nsteps < 0 || !finite_pos(dt) || every < 1 || n_traj < 1 || !cot || !out) return SHGB_EINVAL;
  if (!adjoint_supported(md, st)) return SHGB_EUNSUPPORTED;
  if (shgb_checkpoint_bytes(st->n_beams, st->m, nsteps, every) > 0 && !ckpt) return SHGB_EINVAL;
  if (!work || work_bytes < shgb_population_adjoint_workspace(st->n_beams, st->m, every)) return SHGB_EWORKSPACE;
  if (st->m == 2)
    return hip_status(launch_adjoint_m2(md, *st, ckpt, nsteps, dt, seed, every, cot, n_traj, out, work,
                                        (hipStream_t)stream));
  return hip_status(launch_adjoint_wave(md, *st, ckpt, nullptr, nsteps, dt, seed, every, cot, n_traj, out, work,
                                        (hipStream_t)stream));
}

int64_t shgb_batch_table_bytes(int32_t n_inst) {
  if (n_inst < 1) return -1;
  return (int64_t)n_inst * (int64_t)sizeof(BatchItem);
}

int shgb_batch_prepare(const shgb_model *models, const shgb_state *states, const uint64_t *seeds, int32_t n_inst,
                       const shgb_batch_config *cfg, void *host_table, int64_t table_bytes, shgb_batch *batch) {
  if (!models || !states || !seeds || !cfg || !host_table || !batch || n_inst < 1) return SHGB_EINVAL;
  if (table_bytes < shgb_batch_table_bytes(n_inst)) return SHGB_EINVAL;
  if ((cfg->waves_per_block != 2 && cfg->waves_per_block != 4) || cfg->blocks_per_cu < 1 ||
      cfg->blocks_per_cu > 16 || cfg->tiles_per_grab < 1)
    return SHGB_EINVAL;
  BatchItem *items = (BatchItem *)host_table;
  int64_t tiles = 0;
  int d = 0, prec = 0;
  for (int i = 0; i < n_inst; ++i) {
    DevModel md;
    int rc = to_dev_model(&models[i], md);
    if (rc) return rc;
    if (md.kind != SHGB_MODEL_QCLE) return SHGB_EUNSUPPORTED;
    if ((rc = check_state(&states[i], md))) return rc;
    if (i == 0) {
      d = md.d;
      prec = states[i].precision;
      if (d != 1 && !step_wave_supported(d)) return SHGB_EUNSUPPORTED;
    } else if (md.d != d || states[i].precision != prec) {
      return SHGB_EINVAL;
    }
    const int64_t tb = d == 1 ? m2_tile_beams(cfg->waves_per_block) : wave_tile_beams(d, cfg->waves_per_block);
    BatchItem &it = items[i];
    std::memset(&it, 0, sizeof(it));
    it.md = md;
    it.tr = prec == SHGB_MIXED ? (void *)states[i].f32 : (void *)states[i].f64;
    it.sc = scalar_block(states[i]);
    it.comp = states[i].comp;
    it.nhop = states[i].nhop;
    it.n = states[i].n_beams;
    it.ld = states[i].ld;
    it.gid0 = states[i].beam_id_offset;
    it.seed = seeds[i];
    it.tile0 = tiles;
    it.tiles = (it.n + tb - 1) / tb;
    tiles += it.tiles;
  }
  batch->n_inst = n_inst;
  batch->d = d;
  batch->precision = prec;
  batch->kind = SHGB_MODEL_QCLE;
  batch->total_tiles = tiles;
  batch->cfg = *cfg;
  batch->table = nullptr;
  return SHGB_OK;
}

int shgb_step_batched(const shgb_batch *batch, int32_t nsteps, double dt, void *work, int64_t work_bytes,
                      uint64_t *diag, void *stream) {
  if (!batch || batch->n_inst < 1 || nsteps < 0 || !finite_pos(dt)) return SHGB_EINVAL;
  if (!work || work_bytes < SHGB_BATCH_WORK_BYTES) return SHGB_EINVAL;
  const shgb_batch_config &cfg = batch->cfg;
  if ((cfg.waves_per_block != 2 && cfg.waves_per_block != 4) || cfg.blocks_per_cu < 1 || cfg.blocks_per_cu > 16 ||
      cfg.tiles_per_grab < 1 || batch->total_tiles < 0)
    return SHGB_EINVAL;
  if (batch->kind != SHGB_MODEL_QCLE || batch->d < 1 || batch->d > SHGB_MAX_D ||
      (batch->precision != SHGB_FP64 && batch->precision != SHGB_MIXED))
    return SHGB_EINVAL;
  if (batch->total_tiles == 0 || nsteps == 0) return SHGB_OK;
  if (!batch->table) return SHGB_EINVAL;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return SHGB_EHIP;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long *queue = (unsigned long long *)work;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, queue);
  const int blocks = cus * cfg.blocks_per_cu;
  const bool mx = batch->precision == SHGB_MIXED;
  const BatchItem *items = (const BatchItem *)batch->table;
  hipError_t e;
  if (batch->d == 1)
    e = launch_step_m2_batched(mx, cfg.waves_per_block, items, batch->n_inst, batch->total_tiles, cfg.tiles_per_grab,
                               blocks, nsteps, dt, queue, diag, s);
  else
    e = launch_step_wave_batched(batch->d, mx, cfg.waves_per_block, items, batch->n_inst, batch->total_tiles,
                                 cfg.tiles_per_grab, blocks, nsteps, dt, queue, diag, s);
  return hip_status(e);
}

int shgb_philox(uint64_t seed, const uint64_t *counters, uint64_t *out, int64_t n, void *stream) {
  if (n < 0 || (n > 0 && (!counters || !out))) return SHGB_EINVAL;
  return hip_status(launch_philox(seed, counters, out, n, (hipStream_t)stream));
}

const char *shgb_strerror(int code) {
  switch (code) {
    case SHGB_OK: return "ok";
    case SHGB_EINVAL: return "invalid argument";
    case SHGB_EUNSUPPORTED: return "unsupported model or dimension";
    case SHGB_EHIP: return "HIP launch or runtime error";
    case SHGB_EWORKSPACE: return "workspace too small";
    default: return "unknown error";
  }
}

int32_t shgb_version(void) { return 1; }

void shgb_abi_sizes(int64_t *sizes) {
  if (!sizes) return;
  sizes[0] = (int64_t)sizeof(shgb_model);
  sizes[1] = (int64_t)sizeof(shgb_state);
  sizes[2] = (int64_t)sizeof(shgb_init_spec);
  sizes[3] = (int64_t)sizeof(shgb_batch_config);
  sizes[4] = (int64_t)sizeof(shgb_batch);
}

}  // extern "C"
