"""Populations as differentiable functions of the model and initial-data
parameters (torch.autograd), through the pathwise tangent kernel.

``population(theta, cfg, component)`` returns the population of one
component after the configured run, as a function of
theta = (A, B, C, D, p_mean); its backward multiplies the incoming gradient
by the derivative shgb_population_tangent computes (hop sequences frozen,
see include/shgb.h).  The forward pass samples a fresh ensemble with the
configured seed each call, so repeated calls with one theta agree exactly.
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
    """(sums, derivatives) for the run of cfg at theta: sums (4, 2) = (Re, Im) of sum c per
    component; derivatives (5, 4, 2) along each theta_j.  Host float64 tensors."""
    mdl = _model(theta, cfg)
    st = shgb.State(cfg["n_beams"], 2 * cfg["d"], device=device)
    shgb.init_beams(mdl, _spec(theta, cfg), st, cfg["seed"])
    out = shgb.population_tangent(mdl, st, cfg["nsteps"], cfg["dt"], cfg["seed"]).cpu()
    return out[0, :, 0:2].clone(), out[:, :, 2:4].clone()


class _Population(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, cfg, component):
        sums, deriv = population_and_tangent(theta.detach().cpu().tolist(), cfg)
        n = cfg["n_beams"]
        ctx.save_for_backward(deriv[:, component, 0].to(theta) / n)
        return (sums[component, 0] / n).to(theta)

    @staticmethod
    def backward(ctx, grad):
        (g,) = ctx.saved_tensors
        return grad * g, None, None


def population(theta, cfg, component=0):
    """Re of the population of `component` (0 = upper surface) after the run of cfg, differentiable
    in theta = (A, B, C, D, p_mean) (a float64 tensor of 5)."""
    return _Population.apply(theta, cfg, component)
