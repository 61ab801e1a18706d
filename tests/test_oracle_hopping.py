"""Pins for the oracle's hopping algorithm (Sec. 2.2 and Sec. 2.4 steps 2-7).

P3  x-independent coefficients (alpha = 0, constant beta_l, constant complex
    gamma with nonzero diagonal): the system is du/dt = (i diag(beta)/eps + Gamma) u
    for every x, whose solution is a matrix exponential (Sec. 2.2 eq:tilde_gamma
    with the diagonal kept).  The SHGB estimator's mean must match it within
    its standard error; with constant rates the linearly interpolated hop
    times are exactly exponential and the destinations follow |gamma_jl|.
"""

import math

import numpy as np
from scipy import linalg, stats

from oracle import models, observables, philox, shgb

B0 = np.array([0.3, -0.5, 1.1])
GAM = np.array([[-0.2 + 0.1j, 0.4 - 0.3j, 0.2j],
                [0.7 + 0.2j, 0.1 - 0.3j, -0.5],
                [0.3 - 0.6j, 0.9, -0.4 + 0.2j]])
EPS = 0.5


def xindep_ensemble(n, comp0=0, seed=3):
    ens = shgb.Ensemble(n, 2, 3)
    ens.gid[:] = np.arange(n, dtype=np.uint64)
    ens.M[:] = np.eye(2)
    ens.A[:] = 1.0 / (2 * math.pi * EPS)      # each beam integrates to one
    ens.comp[:] = comp0
    for b in range(n):
        ens.E[b] = shgb.threshold(philox.u01(philox.block(seed, b, 0, philox.TAG_HOP)[1]))
    return ens


def test_P3_populations_match_matrix_exponential():
    model = models.LinQuad.xindep(B0, GAM)
    n, T, steps, seed = 20000, 1.0, 10, 3
    ens = xindep_ensemble(n, seed=seed)
    shgb.advance(model, ens, steps, T / steps, seed)
    mean, se = observables.population_mean_se(observables.populations(ens, EPS), n)
    exact = linalg.expm(T * (1j * np.diag(B0) / EPS + GAM))[:, 0]
    for i in range(3):
        assert abs(mean[i].real - exact[i].real) < 4 * se[i].real + 1e-3, (i, mean, exact, se)
        assert abs(mean[i].imag - exact[i].imag) < 4 * se[i].imag + 1e-3, (i, mean, exact, se)
    # a dropped phase factor or weight is far outside these bands
    assert np.abs(exact).min() > 0.05


def test_P3_waiting_times_and_destinations():
    model = models.LinQuad.xindep(B0, GAM)
    n, T, steps, seed = 6000, 1.0, 7, 11
    ens = xindep_ensemble(n, seed=seed)
    shgb.advance(model, ens, steps, T / steps, seed)
    R0 = abs(GAM[1, 0]) + abs(GAM[2, 0])
    first = [log[0] for log in ens.hop_log if log]
    t1 = np.array([h[2] for h in first])
    # censored at T: compare the conditional law on [0, T]
    cdf = lambda t: (1 - np.exp(-R0 * t)) / (1 - math.exp(-R0 * T))
    assert stats.kstest(t1, cdf).pvalue > 1e-3
    assert abs(len(first) / n - (1 - math.exp(-R0 * T))) < 4 * math.sqrt(0.25 / n)
    dest = np.array([h[1] for h in first])
    p1 = abs(GAM[1, 0]) / R0
    k = (dest == 1).sum()
    assert abs(k / len(dest) - p1) < 4 * math.sqrt(p1 * (1 - p1) / len(dest))


# coupling column of component 0 with rates |gamma_10| : |gamma_20| = 9 : 1 (complex entries)
GAM_UNEQUAL = np.array([[0.0, 0.1, 0.2], [0.9 * np.exp(0.3j), 0.0, 0.1], [0.1j, 0.3, 0.0]])


def forced_hop_destinations(shgb_mod, n=5000, seed=21):
    """Destinations of n hops forced at once from component 0 (hop_event of ``shgb_mod``)."""
    model = models.LinQuad.xindep(B0, GAM_UNEQUAL)
    ens = xindep_ensemble(n, comp0=0, seed=seed)
    ens.E[:] = 0.0
    shgb_mod.hop_event(model, ens, np.arange(n), seed)
    return ens.comp.copy()


def test_destinations_follow_unequal_rates():
    """Sec. 2.4 step 5: the destination j is drawn with probability |gamma_j0| / sum_k |gamma_k0|
    (here 0.9 and 0.1; binomial band of 4 SE)."""
    dest = forced_hop_destinations(shgb)
    assert np.isin(dest, [1, 2]).all()
    p1, n = 0.9, dest.size
    assert abs((dest == 1).mean() - p1) < 4 * math.sqrt(p1 * (1 - p1) / n)


def test_forced_hop_and_weight_bookkeeping():
    """A threshold at or below Lam hops at once; phase and weight follow gamma."""
    model = models.LinQuad.xindep(B0, GAM)
    ens = xindep_ensemble(4, comp0=1, seed=5)
    ens.Lam[:] = 0.25
    ens.E[:] = 0.0
    shgb.hop_event(model, ens, np.arange(4), seed=5)
    for b in range(4):
        j = ens.comp[b]
        assert j != 1
        np.testing.assert_allclose(ens.phase[b], GAM[j, 1] / abs(GAM[j, 1]), rtol=1e-15)
        assert ens.logw[b] == 0.25 and ens.Lam[b] == 0.0 and ens.nhop[b] == 1
        w = philox.block(5, b, 1, philox.TAG_HOP)
        assert abs(ens.E[b] + math.log(1.0 - philox.u01(w[1]))) <= 4e-16 * ens.E[b]
    # inside advance_interval: E = 0 with Lam = 0 -> theta = 0 hop at the interval start
    ens2 = xindep_ensemble(3, comp0=2, seed=5)
    ens2.E[:] = 0.0
    S_before = ens2.S.copy()
    shgb.advance_interval(model, ens2, 0.1, seed=5)
    assert (ens2.nhop >= 1).all()
    assert all(log[0][2] == 0.0 for log in ens2.hop_log)
    # the whole interval is then integrated on the new component
    np.testing.assert_allclose(ens2.S - S_before, 0.1 * B0[ens2.comp], rtol=1e-13)


def test_hop_cap_bounds_work():
    """Enormous rates: at most HOP_CAP hops per interval, overflow counted."""
    model = models.LinQuad.xindep(B0, GAM * 1e6)
    ens = xindep_ensemble(5, seed=2)
    shgb.advance_interval(model, ens, 0.5, seed=2)
    assert (ens.nhop == shgb.HOP_CAP).all()
    assert (ens.cap_overflow == 1).all()
