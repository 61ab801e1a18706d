"""Planted mistakes: each plausible error in the oracle's beam ODEs, RK4 and
hopping code makes one of its pins fail.

The source of oracle/shgb.py is loaded with one textual change into a fresh
module (in memory, on the CPU) and the checks of two pins run against it:
P1 (closed-form propagation of a linear-quadratic beam, tests/test_oracle_gb.py)
for the right-hand side of eq:shgb_odes and the RK4 step, and P3 (x-independent
system: populations against the matrix exponential, first hop times against
the exponential law, destinations of forced hops against unequal rates,
tests/test_oracle_hopping.py) and the QCLE weight invariant
Re omega = 2 |theta(q_T) - theta(q_0)| (tests/test_oracle_qcle.py) for the hop
bookkeeping of Sec. 2.4.  The unchanged source, loaded the same way, passes
every check.  The same is done for oracle/observables.py against its pins:
the beam integral against two-dimensional quadrature, the field summed on a
fine grid against the populations, and the field's momentum expectation
against P; and for the QCLE coefficients of oracle/models.py against the
energies of numpy.linalg.eigvalsh and the derivative of the eigenvector angle;
and for the initial sampling of oracle/sampling.py against the law of the
centres and the unit beam integral, and its bath modes against the ground
state of each harmonic mode (energy, its kinetic and potential parts,
q-p correlation, normality).
"""

import math
import types

import numpy as np
import pytest
from scipy import linalg, stats

import oracle.models as models_base
import oracle.observables as obs_base
import oracle.sampling as sampling_base
import oracle.shgb as base
from oracle import models, observables, sampling

import test_oracle_gb as gb
import test_oracle_hopping as hop
import test_oracle_model as model_pins
import test_oracle_observables as obs_pins
import test_oracle_qcle as qcle


def load(old=None, new=None, original=base):
    src = open(original.__file__).read()
    if old is not None:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    mod = types.ModuleType(original.__name__ + "_planted")
    mod.__file__, mod.__package__ = original.__file__, "oracle"
    exec(compile(src, original.__file__, "exec"), mod.__dict__)
    return mod


def p1_error(mod, m=2, n=80, T=1.5):
    """Max error of a beam after n RK4 steps against its closed form (the P1 bar at n = 80: 1e-6)."""
    model, ens = gb.random_linquad(m, seed=m), gb.one_beam(m, seed=m)
    XT, PT, ZT, ST, AT = gb.exact_beam(model, ens, T)
    e = ens.subset([0])
    for _ in range(n):
        mod.advance_interval(model, e, T / n, seed=1)
    return max(np.abs(e.X[0] - XT).max(), np.abs(e.P[0] - PT).max(), np.abs(e.M[0] + 1j * e.N[0] - ZT).max(),
               abs(e.S[0] - ST), abs(e.A[0] - AT))


def p3_run(mod, n=4000, T=1.0, steps=10, seed=3):
    model = models.LinQuad.xindep(hop.B0, hop.GAM)
    ens = hop.xindep_ensemble(n, seed=seed)
    mod.advance(model, ens, steps, T / steps, seed)
    return model, ens


def p3_population_excess(mod, n=4000, T=1.0):
    """Largest |mean - exact| over the P3 band 4 SE + 1e-3 (the pin passes below 1)."""
    _, ens = p3_run(mod, n, T)
    mean, se = observables.population_mean_se(observables.populations(ens, hop.EPS), n)
    exact = linalg.expm(T * (1j * np.diag(hop.B0) / hop.EPS + hop.GAM))[:, 0]
    return max(max(abs(mean[i].real - exact[i].real) / (4 * se[i].real + 1e-3),
                   abs(mean[i].imag - exact[i].imag) / (4 * se[i].imag + 1e-3)) for i in range(3))


def p3_first_hop_pvalue(mod, n=4000, T=1.0):
    """KS p-value of the first hop times against the censored exponential law (the pin: > 1e-3)."""
    _, ens = p3_run(mod, n, T, steps=7, seed=11)
    R0 = abs(hop.GAM[1, 0]) + abs(hop.GAM[2, 0])
    t1 = np.array([log[0][2] for log in ens.hop_log if log])
    return stats.kstest(t1, lambda t: (1 - np.exp(-R0 * t)) / (1 - math.exp(-R0 * T))).pvalue


def qcle_weight_error(mod, n=100, nsteps=700):
    """Largest |logw + Lam - 2 |theta(q_T) - theta(q_0)|| relative to the largest angle term, on
    the QCLE ensemble of tests/test_oracle_qcle.py (the pin: 1e-7 relative)."""
    mdl = models.QCLE(**qcle.PAR)
    ens = sampling.init_beams(mdl, n, qcle.EPS, 99, -2.5, 0.3, "normal", 30.0, 1.0, 1)
    th0 = mdl.mixing_angle(ens.X[:, 0])
    mod.advance(mdl, ens, nsteps, 0.5, 99)
    ref = 2 * np.abs(mdl.mixing_angle(ens.X[:, 0]) - th0)
    return np.abs(ens.logw + ens.Lam - ref).max() / ref.max()


def test_unchanged_source_passes_every_check():
    mod = load()
    assert p1_error(mod) < 1e-6
    assert p3_population_excess(mod) < 1.0
    assert p3_first_hop_pvalue(mod) > 1e-3
    assert qcle_weight_error(mod) < 1e-7


ODE_MISTAKES = {
    "dP: sign of the J^T P term": ('- np.einsum("nab,nb->na", Jt, P)', '+ np.einsum("nab,nb->na", Jt, P)'),
    "dM: J and J^T exchanged": ("dM = -M @ J - Jt @ M", "dM = -M @ Jt - J @ M"),
    "dN: sign of Hess beta": ("- model.hess_beta(X, comp) - N @ J", "+ model.hess_beta(X, comp) - N @ J"),
    "dS: sign of beta": ("dS = model.beta(X, comp)", "dS = -model.beta(X, comp)"),
    "dA: gamma_ll dropped": ("dA = G[idx, comp, comp] * A", "dA = 0.0 * A"),
    "RK4: weights of k3 and k4 exchanged": ("(b1 + 2.0 * b2 + 2.0 * b3 + b4)", "(b1 + 2.0 * b2 + b3 + 2.0 * b4)"),
    "RK4: k3 from k1": ("k3 = rhs(model, comp, _axpy(y, 0.5 * h, k2))", "k3 = rhs(model, comp, _axpy(y, 0.5 * h, k1))"),
}


@pytest.mark.parametrize("name", list(ODE_MISTAKES))
def test_P1_catches_planted_ode_mistake(name):
    err = p1_error(load(*ODE_MISTAKES[name]))
    assert err > 1e-4, (name, err)      # 100x the pin's bar


HOP_MISTAKES = {
    "phase jump conjugated": ("ens.phase[b] * (col[dest] / abs(col[dest]))",
                              "ens.phase[b] * (col[dest].conjugate() / abs(col[dest]))"),
    "weight update dropped": ("ens.logw[b] += ens.Lam[b]", "ens.logw[b] += 0.0"),
    "coupling row instead of column": ("col = [complex(g) for g in G[t, :, l]]",
                                       "col = [complex(g) for g in G[t, l, :]]"),
}


@pytest.mark.parametrize("name", list(HOP_MISTAKES))
def test_P3_catches_planted_hop_mistake(name):
    excess = p3_population_excess(load(*HOP_MISTAKES[name]))
    assert excess > 2.0, (name, excess)   # twice the pin's band


def test_P3_waiting_times_catch_out_rate_with_gamma_ll():
    mod = load("out_rate = np.abs(G[idx, :, comp]).sum(1) - np.abs(G[idx, comp, comp])",
               "out_rate = np.abs(G[idx, :, comp]).sum(1)")
    assert p3_first_hop_pvalue(mod) < 1e-4


def test_destination_pin_catches_uniform_destinations():
    mod = load("            for j in order:\n                C = C + abs(col[j])\n                if U * R < C:",
               "            for j in order:\n                C = C + R / len(order)\n                if U * R < C:")
    dest = hop.forced_hop_destinations(mod)
    assert abs((dest == 1).mean() - 0.9) > 0.2


def test_QCLE_weight_invariant_catches_Lam_not_reset_at_a_hop():
    # the x-independent populations do not see this one: the estimator's own standard error
    # grows with the overcounted weights and widens the band
    err = qcle_weight_error(load("ens.Lam[b] = 0.0", "ens.Lam[b] = ens.Lam[b]"))
    assert err > 1e-3, err


def test_P3_catches_hop_at_the_end_of_the_trial_step():
    mod = load("theta = np.where(Ec <= L0c, 0.0, (Ec - L0c) / (L1c - L0c))",
               "theta = np.where(Ec <= L0c, 0.0, np.ones_like(Ec))")
    assert p3_first_hop_pvalue(mod) < 1e-6


def dblquad_error(obs, seed=0, eps=0.4):
    """Relative error of the closed-form beam integral against quadrature (the pin: 1e-8)."""
    e = obs_pins.random_beam(2, np.random.default_rng(seed), eps)
    got = obs.beam_integrals(e, eps)[0]
    return abs(got - obs_pins.dblquad_integral(e, eps)) / max(1.0, abs(got))


def grid_error(obs):
    """Largest |grid integral of the field - population| relative to the largest population
    (the pin: 1e-9)."""
    integral, pops = obs_pins.grid_integral_and_populations(obs)
    ref = pops[:, 0] + 1j * pops[:, 1]
    return np.abs(integral - ref).max() / np.abs(ref).max()


def test_unchanged_observables_pass_their_checks():
    obs = load(original=obs_base)
    assert dblquad_error(obs) < 1e-8 and grid_error(obs) < 1e-9 and momentum_error(obs) < 1e-9


OBSERVABLE_MISTAKES = {
    "det(Z)^(+1/2)": ("/ sqrt_det * np.exp(-quad / (2.0 * eps))", "* sqrt_det * np.exp(-quad / (2.0 * eps))"),
    "sign of P^T Z^-1 P": ("sqrt_det * np.exp(-quad / (2.0 * eps))", "sqrt_det * np.exp(quad / (2.0 * eps))"),
    "conjugate Z in the integral": ("    Z = ens.M + 1j * ens.N\n    lam = np.linalg.eigvals(Z)",
                                    "    Z = ens.M - 1j * ens.N\n    lam = np.linalg.eigvals(Z)"),
    "phase exp(i S / eps) dropped from the integral": (
        "return beam_weights(ens) * np.exp(1j * ens.S / eps) * gauss", "return beam_weights(ens) * gauss"),
    "field: sign of the linear term": ("np.exp(-quad / (2.0 * eps) + 1j * lin / eps)",
                                       "np.exp(-quad / (2.0 * eps) - 1j * lin / eps)"),
    "field: M instead of Z": ('quad = np.einsum("kqa,kab,kqb->kq", y, Z[sl], y)',
                              'quad = np.einsum("kqa,kab,kqb->kq", y, ens.M[sl], y)'),
}


def momentum_error(obs):
    """Largest |<-i eps grad> - P| of one beam's field (the pin: 1e-9)."""
    e, _, p_mean = obs_pins.field_moments(obs)
    return np.abs(p_mean - e.P[0]).max()


@pytest.mark.parametrize("name", list(OBSERVABLE_MISTAKES))
def test_observable_pins_catch_planted_mistake(name):
    obs = load(*OBSERVABLE_MISTAKES[name], original=obs_base)
    if name == "field: sign of the linear term":
        # the grid integral is even in P and does not see this one; the momentum pin does
        err = momentum_error(obs)
    else:
        err = grid_error(obs) if name.startswith("field") else dblquad_error(obs)
    assert err > 1e-4, (name, err)


def energy_error(mod):
    """Largest relative error of the surface energies against eigvalsh (the pin: 1e-13)."""
    return max(np.abs(E - ref).max() / np.abs(ref).max() for E, ref in model_pins.energy_errors(1, mod))


def test_unchanged_model_passes_its_checks():
    mod = load(original=models_base)
    e_d21, e_ang = model_pins.d21_and_angle_errors(mod)
    assert energy_error(mod) < 1e-13 and e_d21 <= 1e-6 and e_ang < 1e-12


MODEL_MISTAKES = {
    "s without the factor 4 on V12^2": ("s = sp.sqrt((V11 - V22) ** 2 + 4 * V12**2) / 2",
                                        "s = sp.sqrt((V11 - V22) ** 2 + V12**2) / 2"),
    "V22 = +a": ("V11, V22, V12 = a, -a, self.C", "V11, V22, V12 = a, a, self.C"),
    "d21 with the opposite sign": (
        "d21 = ((V11 - V22) * sp.diff(V12, q) - V12 * sp.diff(V11 - V22, q)) / (",
        "d21 = (V12 * sp.diff(V11 - V22, q) - (V11 - V22) * sp.diff(V12, q)) / ("),
    "d21 denominator without the factor 4": ("/ (\n            (V11 - V22) ** 2 + 4 * V12**2)",
                                             "/ (\n            (V11 - V22) ** 2 + V12**2)"),
}


@pytest.mark.parametrize("name", list(MODEL_MISTAKES))
def test_model_pins_catch_planted_mistake(name):
    mod = load(*MODEL_MISTAKES[name], original=models_base)
    err = model_pins.d21_and_angle_errors(mod)[0] if name.startswith("d21") else energy_error(mod)
    assert err > 1e-4, (name, err)


def test_unchanged_sampling_passes_its_checks():
    err_c, z_q, err_std, p_ks = qcle.initial_law(load(original=sampling_base))
    assert err_c < 1e-13 and z_q < 4.0 and err_std < 0.0134 and p_ks > 1e-3


SAMPLING_MISTAKES = {
    "A0 = (2 pi eps)^(+m/2)": ("ens.A[:] = (2.0 * math.pi * eps) ** (-m / 2.0)",
                               "ens.A[:] = (2.0 * math.pi * eps) ** (m / 2.0)"),
    "q_std not applied": ("x[0] = q_mean + q_std * normal(seed, gid, 0)", "x[0] = q_mean + normal(seed, gid, 0)"),
    "uniform law on [p_a, p_a + p_b)": ("x[d] = p_a + (p_b - p_a) * uniform(seed, gid, d)",
                                        "x[d] = p_a + p_b * uniform(seed, gid, d)"),
}


@pytest.mark.parametrize("name", list(SAMPLING_MISTAKES))
def test_sampling_pin_catches_planted_mistake(name):
    err_c, z_q, err_std, p_ks = qcle.initial_law(load(*SAMPLING_MISTAKES[name], original=sampling_base))
    assert err_c > 1e-3 or z_q > 8.0 or err_std > 0.05 or p_ks < 1e-6, name


def test_unchanged_sampling_passes_the_bath_law():
    z_energy, z_parts, corr, p_ks = qcle.bath_law(load(original=sampling_base))
    assert z_energy < 4.0 and z_parts < 4.0 and corr < 4.0 and p_ks > 1e-3


BATH_MISTAKES = {
    "mass swapped between the two widths": (
        "x[k] = math.sqrt(eps / (2.0 * model.mass * w)) * normal(seed, gid, k)\n"
        "            x[d + k] = math.sqrt(eps * model.mass * w / 2.0) * normal(seed, gid, d + k)",
        "x[k] = math.sqrt(eps * model.mass / (2.0 * w)) * normal(seed, gid, k)\n"
        "            x[d + k] = math.sqrt(eps * w / (2.0 * model.mass)) * normal(seed, gid, d + k)"),
    "frequency swapped between the two widths": (
        "x[k] = math.sqrt(eps / (2.0 * model.mass * w)) * normal(seed, gid, k)\n"
        "            x[d + k] = math.sqrt(eps * model.mass * w / 2.0) * normal(seed, gid, d + k)",
        "x[k] = math.sqrt(eps * w / (2.0 * model.mass)) * normal(seed, gid, k)\n"
        "            x[d + k] = math.sqrt(eps * model.mass / (2.0 * w)) * normal(seed, gid, d + k)"),
    "factor 2 dropped from the position width": (
        "x[k] = math.sqrt(eps / (2.0 * model.mass * w))", "x[k] = math.sqrt(eps / (model.mass * w))"),
    "variance used as the momentum width": (
        "x[d + k] = math.sqrt(eps * model.mass * w / 2.0) * normal", "x[d + k] = (eps * model.mass * w / 2.0) * normal"),
    "position and momentum from the same normal": (
        "x[d + k] = math.sqrt(eps * model.mass * w / 2.0) * normal(seed, gid, d + k)",
        "x[d + k] = math.sqrt(eps * model.mass * w / 2.0) * normal(seed, gid, k)"),
    "bath frequencies out by one mode": ("w = model.bath_omega[k - 1]", "w = model.bath_omega[k % (d - 1)]"),
}


@pytest.mark.parametrize("name", list(BATH_MISTAKES))
def test_bath_law_catches_planted_mistake(name):
    z_energy, z_parts, corr, p_ks = qcle.bath_law(load(*BATH_MISTAKES[name], original=sampling_base))
    assert z_energy > 8.0 or z_parts > 8.0 or corr > 8.0 or p_ks < 1e-6, (name, z_energy, z_parts, corr, p_ks)


def p1_error_rk3(mod, m=2, n=160, T=1.5):
    """Max error of a beam after n third-order steps against its closed form (the order-3 pin: 1e-4)."""
    model, ens = gb.random_linquad(m, seed=m), gb.one_beam(m, seed=m)
    XT, PT, ZT, ST, AT = gb.exact_beam(model, ens, T)
    e = ens.subset([0])
    for _ in range(n):
        mod.advance_interval(model, e, T / n, seed=1, scheme="rk3")
    return max(np.abs(e.X[0] - XT).max(), np.abs(e.P[0] - PT).max(), np.abs(e.M[0] + 1j * e.N[0] - ZT).max(),
               abs(e.S[0] - ST), abs(e.A[0] - AT))


def rk3_order_check(mod):
    """(error at 160 steps, error ratio from 80 to 160 steps): the pin wants < 1e-4 and about 8."""
    e80, e160 = p1_error_rk3(mod, n=80), p1_error_rk3(mod, n=160)
    return e160, e80 / e160


def test_unchanged_source_passes_the_order3_check():
    err, ratio = rk3_order_check(load())
    assert err < 1e-4 and 6.5 < ratio < 9.5


RK3_MISTAKES = {
    "RK3: middle weight 2 instead of 4": ("(b1 + 4.0 * b2 + b3)", "(b1 + 2.0 * b2 + b3)"),
    "RK3: third stage at y + h k2": ("k3 = rhs(model, comp, _axpy(_axpy(y, -h, k1), 2.0 * h, k2))",
                                     "k3 = rhs(model, comp, _axpy(y, h, k2))"),
    "RK3: second stage at the full step": ("k2 = rhs(model, comp, _axpy(y, 0.5 * h, k1))\n    k3 = rhs(model, comp, _axpy(_axpy(",
                                           "k2 = rhs(model, comp, _axpy(y, h, k1))\n    k3 = rhs(model, comp, _axpy(_axpy("),
}


@pytest.mark.parametrize("name", list(RK3_MISTAKES))
def test_P1_order3_catches_planted_rk3_mistake(name):
    err, ratio = rk3_order_check(load(*RK3_MISTAKES[name]))
    assert err > 1e-3 or not 6.5 < ratio < 9.5, (name, err, ratio)
