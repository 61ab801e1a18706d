"""Populations as differentiable functions of the model and initial-data
parameters (torch.autograd), through the reverse-mode (adjoint) kernel.

``populations(theta, cfg)`` returns the (Re, Im) population means of the four
components after the configured run, a (4, 2) float64 device tensor, as a
function of theta = (A, B, C, D, p_mean).  Its forward pass samples the
ensemble with the configured seed (repeated calls with one theta agree
exactly), steps it with checkpoints every ``every`` intervals and forms the
means on the device; its backward pass launches the reverse sweep
(shgb_population_adjoint) with the incoming gradient as the cotangent, one
sweep for all five parameters (hop sequences frozen, see include/shgb.h).
For d > 1 the forward pass can keep every interval's stage records in device
memory (shgb_step_recorded) so that the backward pass need not run the
segments again (shgb_population_adjoint_recorded): ``keep_records`` True or
False, or None to keep them when they take at most half of the free device
memory.  Both give the same gradient.
``population_and_tangent`` gives the same derivative by forward (tangent)
propagation, one pass per parameter: the check of the adjoint.
"""

import torch

from . import shgb


def _model(theta, cfg):
    A, B, C, D = (float(x) for x in theta[:4])
    return shgb.make_model(cfg["d"], cfg["mass"], cfg["eps"], A, B, C, D, cfg.get("lam", 0.0),
                           cfg.get("bath_omega", ()))


def _spec(theta, cfg):
    shift = float(theta[4]) - theta_of(cfg)[4]    # p_mean moves the initial momentum law as a whole
    if cfg["p_dist"] == "normal":
        return shgb.make_init_spec(cfg["q_mean"], cfg["q_std"], "normal", cfg["p_a"] + shift, cfg["p_b"],
                                   cfg["comp0"])
    return shgb.make_init_spec(cfg["q_mean"], cfg["q_std"], "uniform", cfg["p_a"] + shift, cfg["p_b"] + shift,
                               cfg["comp0"])


def theta_of(cfg):
    """theta = (A, B, C, D, p_mean) of a workload config; p_mean is the centre of the p1 law."""
    p_mean = cfg["p_a"] if cfg["p_dist"] == "normal" else 0.5 * (cfg["p_a"] + cfg["p_b"])
    return [cfg["A"], cfg["B"], cfg["C"], cfg["D"], p_mean]


def population_and_tangent(theta, cfg, device="cuda"):
    """(sums, derivatives) for the run of cfg at theta by the tangent kernel: sums (4, 2) = (Re, Im)
    of sum c per component; derivatives (5, 4, 2) along each theta_j.  Host float64 tensors."""
    mdl = _model(theta, cfg)
    st = shgb.State(cfg["n_beams"], 2 * cfg["d"], device=device)
    shgb.init_beams(mdl, _spec(theta, cfg), st, cfg["seed"])
    out = shgb.population_tangent(mdl, st, cfg["nsteps"], cfg["dt"], cfg["seed"]).cpu()
    return out[0, :, 0:2].clone(), out[:, :, 2:4].clone()


def _keep(cfg, every, keep_records):
    if cfg["d"] == 1:
        return False                      # the one-dimensional adjoint has no kept-records form
    if keep_records is not None:
        return bool(keep_records)
    need = shgb.record_bytes(cfg["n_beams"], 2 * cfg["d"], cfg["nsteps"], every)
    free, _ = torch.cuda.mem_get_info()
    return need <= free // 2


class _Populations(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, cfg, every, keep_records):
        th = theta.detach().cpu().tolist()
        mdl = _model(th, cfg)
        st = shgb.State(cfg["n_beams"], 2 * cfg["d"])
        shgb.init_beams(mdl, _spec(th, cfg), st, cfg["seed"])
        recs = None
        if _keep(cfg, every, keep_records):
            ckpt, recs = shgb.step_recorded(mdl, st, cfg["nsteps"], cfg["dt"], cfg["seed"], every=every)
        else:
            ckpt = shgb.step_checkpointed(mdl, st, cfg["nsteps"], cfg["dt"], cfg["seed"], every=every)
        stats = shgb.population_stats(shgb.populations(mdl, st), cfg["n_beams"])
        ctx.run = (mdl, st, ckpt, recs, cfg, every)
        ctx.theta_like = (theta.dtype, theta.device)
        return stats[:, 0:2].contiguous()

    @staticmethod
    def backward(ctx, grad):
        mdl, st, ckpt, recs, cfg, every = ctx.run
        cot = grad.to(dtype=torch.float64).contiguous().view(-1)
        if recs is not None:
            out = shgb.population_adjoint_recorded(mdl, st, ckpt, recs, cfg["nsteps"], cfg["dt"], cfg["seed"], cot,
                                                   cfg["n_beams"], every=every)
        else:
            out = shgb.population_adjoint(mdl, st, ckpt, cfg["nsteps"], cfg["dt"], cfg["seed"], cot,
                                          cfg["n_beams"], every=every)
        dtype, device = ctx.theta_like
        return out[:5].to(dtype=dtype, device=device), None, None, None


def populations(theta, cfg, every=100, keep_records=None):
    """(Re, Im) population means of the four components after the run of cfg, a (4, 2) device
    tensor, differentiable in theta = (A, B, C, D, p_mean) (a float64 tensor of 5)."""
    return _Populations.apply(theta, cfg, every, keep_records)


def population(theta, cfg, component=0, every=100, keep_records=None):
    """Re of the population of `component` (0 = upper surface), differentiable in theta."""
    return populations(theta, cfg, every, keep_records)[component, 0]
