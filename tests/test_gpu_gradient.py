"""Pathwise derivative of the populations (QCLE, m = 2 and the harmonic-bath
model with m = 2d > 2) with respect to theta = (A, B, C, D, p_mean), hop
sequences frozen.

The tangent kernel is checked against central differences of the FP64 GPU
path (Richardson-extrapolated over h and h/2: the phase S/eps makes the
third derivative in p_mean large) and of the oracle, both under common
random numbers and with the hop sequences of the shifted runs checked
identical (otherwise the difference quotient measures a jump, not the
derivative); and the torch.autograd wrapper (whose backward is the reverse-mode kernel)
returns the tangent's derivative.
"""

import numpy as np
import pytest
import torch

from oracle import observables, sampling, shgb as oshgb
from paper_1703_06116_amd import gradient, workloads

from _parity import gpu_model, gpu_spec, oracle_model

pytestmark = pytest.mark.gpu


def crossing_cfg(n, nsteps, d=1, **kw):
    if d == 1:
        return workloads.config("qcle1d_1e4", n_beams=n, nsteps=nsteps, q_mean=-2.5, q_std=0.3, p_a=30.0, **kw)
    return workloads.config("qcle12d_2p18", d=d, bath_omega=workloads.bath_omega(d), n_beams=n, nsteps=nsteps,
                            q_mean=-2.5, q_std=0.3, p_a=30.0, **kw)


def shifted(cfg, j, h):
    th = gradient.theta_of(cfg)
    th[j] += h
    c = dict(cfg, A=th[0], B=th[1], C=th[2], D=th[3])
    if j == 4:
        c["p_a"] = cfg["p_a"] + h
        if cfg["p_dist"] == "uniform":
            c["p_b"] = cfg["p_b"] + h
    return c


def gpu_fp64_run(gpu, c):
    st = gpu.State(c["n_beams"], 2 * c["d"])
    gpu.init_beams(gpu_model(c), gpu_spec(c), st, c["seed"])
    gpu.step_ensemble(gpu_model(c), st, c["nsteps"], c["dt"], c["seed"])
    sums = gpu.populations(gpu_model(c), st).cpu().numpy()
    return sums[:, 0] + 1j * sums[:, 1], st.nhop.cpu().numpy(), st.comp.cpu().numpy()


@pytest.mark.parametrize("d,p_dist,n,nsteps", [(1, "normal", 2 * 256 + 37, 600), (1, "uniform", 2 * 256 + 37, 600),
                                                (2, "normal", 2 * 128 + 5, 500), (12, "normal", 2 * 64 + 3, 450)])
def test_tangent_matches_gpu_central_differences(gpu, d, p_dist, n, nsteps):
    cfg = crossing_cfg(n, nsteps, d=d, p_dist=p_dist, p_b=1.0 if p_dist == "normal" else 34.0)
    theta = gradient.theta_of(cfg)
    sums, deriv = gradient.population_and_tangent(theta, cfg)
    value = sums[:, 0].numpy() + 1j * sums[:, 1].numpy()
    base, nh0, _ = gpu_fp64_run(gpu, cfg)
    assert np.abs(value - base).max() <= 1e-12 * np.abs(base).sum()     # the tangent run's values
    for j in range(5):
        h = 1e-6 * abs(theta[j])
        fds = []
        for hh in (h, 0.5 * h):
            pp, nhp, cp = gpu_fp64_run(gpu, shifted(cfg, j, hh))
            pm, nhm, cm = gpu_fp64_run(gpu, shifted(cfg, j, -hh))
            assert (nhp == nhm).all() and (cp == cm).all() and (nhp == nh0).all(), f"event flipped for theta_{j}"
            fds.append((pp - pm) / (2 * hh))
        fd = (4.0 * fds[1] - fds[0]) / 3.0          # Richardson: the h^2 term of the quotient cancels
        tan = deriv[j, :, 0].numpy() + 1j * deriv[j, :, 1].numpy()
        scale = np.abs(tan).max()
        assert scale > 0
        assert np.abs(fd - tan).max() <= 1e-5 * scale, (j, fd, tan)


def oracle_populations(c):
    om = oracle_model(c)
    e = sampling.init_beams(om, c["n_beams"], c["eps"], c["seed"], c["q_mean"], c["q_std"], c["p_dist"], c["p_a"],
                            c["p_b"], c["comp0"])
    oshgb.advance(om, e, c["nsteps"], c["dt"], c["seed"])
    p = observables.populations(e, c["eps"])
    return p[:, 0] + 1j * p[:, 1], e.nhop.copy(), e.comp.copy()


@pytest.mark.parametrize("d,n,nsteps", [(1, 48, 300), (12, 24, 400)])
def test_tangent_matches_oracle_central_differences(gpu, d, n, nsteps):
    cfg = crossing_cfg(n, nsteps, d=d)
    theta = gradient.theta_of(cfg)
    _, deriv = gradient.population_and_tangent(theta, cfg)
    for j in range(5):
        h = 1e-6 * abs(theta[j])
        pp, nhp, cp = oracle_populations(shifted(cfg, j, h))
        pm, nhm, cm = oracle_populations(shifted(cfg, j, -h))
        assert (nhp == nhm).all() and (cp == cm).all(), f"event flipped for theta_{j}"
        fd = (pp - pm) / (2 * h)
        tan = deriv[j, :, 0].numpy() + 1j * deriv[j, :, 1].numpy()
        assert np.abs(fd - tan).max() <= 1e-5 * np.abs(tan).max(), (j, fd, tan)


@pytest.mark.parametrize("d", [1, 12])
def test_autograd_backward_is_the_adjoint_and_equals_the_tangent(gpu, d):
    cfg = crossing_cfg(300 if d == 1 else 70, 400, d=d)
    theta = torch.tensor(gradient.theta_of(cfg), dtype=torch.float64, requires_grad=True)
    pop = gradient.population(theta, cfg, component=0)
    pop.backward()
    _, deriv = gradient.population_and_tangent(gradient.theta_of(cfg), cfg)
    tan = deriv[:, 0, 0].numpy() / cfg["n_beams"]
    assert np.abs(theta.grad.numpy() - tan).max() <= 1e-10 * np.abs(tan).max()
    # a second call at the same theta gives the same value (fresh ensemble, same seed)
    assert gradient.population(theta.detach(), cfg).item() == pop.item()
    assert abs(pop.item()) < 5.0      # a Monte Carlo estimate with signed weights, not a probability
    # a cotangent over all four components at once
    theta.grad = None
    w = torch.tensor([[0.3, -1.0], [2.0, 0.5], [-0.7, 0.2], [1.1, -0.4]], dtype=torch.float64, device="cuda")
    (gradient.populations(theta, cfg) * w).sum().backward()
    want = (deriv.numpy() * w.cpu().numpy()[None]).sum((1, 2)) / cfg["n_beams"]
    assert np.abs(theta.grad.numpy() - want).max() <= 1e-10 * np.abs(want).max()
    if d > 1:
        # with the stage records kept or not: bitwise the same gradient
        grads = []
        for keep in (True, False):
            theta.grad = None
            (gradient.populations(theta, cfg, keep_records=keep) * w).sum().backward()
            grads.append(theta.grad.clone())
        assert torch.equal(grads[0], grads[1])


@pytest.mark.parametrize("d", [1, 12])
def test_tangent_leaves_the_state_and_respects_the_mask(gpu, d):
    c = crossing_cfg(257 if d == 1 else 37, 50, d=d)
    mdl = gpu_model(c)
    st = gpu.State(c["n_beams"], 2 * d)
    gpu.init_beams(mdl, gpu_spec(c), st, c["seed"])
    before = st.f64.clone()
    out = torch.full((5, 4, 4), 7.0, dtype=torch.float64, device="cuda")
    diag = gpu.new_diag()
    gpu.population_tangent(mdl, st, c["nsteps"], c["dt"], c["seed"], dirs=[1, 4], out=out, diag=diag)
    assert torch.equal(before, st.f64)
    o = out.cpu().numpy()
    assert (o[[0, 2, 3]] == 7.0).all() and not (o[[1, 4]] == 7.0).all()
    np.testing.assert_array_equal(o[1, :, :2], o[4, :, :2])                 # same values in every pass
    empty = gpu.State(0, 2 * d)
    z = gpu.population_tangent(mdl, empty, 10, 0.5, 1)
    assert (z.cpu().numpy() == 0).all()
