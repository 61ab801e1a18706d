"""QCLE invariants of the oracle ensemble (Sec. 2.1 Proposition, Sec. 3.3).

* tr J = 0 (Hamiltonian flow), so det M is constant and M stays symmetric
  positive definite (the proposition of Sec. 2.1 with B1 = 0).
* The total out-rate is 2|kappa| = 2|d theta/dt| on every component (theta the
  mixing angle), so along a trajectory with monotone q1, Re omega(T) =
  logw + Lam = 2 |theta(q1(T)) - theta(q1(0))|, whatever the hops were.
* Initial sampling: every beam integrates to one, all on the lower surface.
* Statistical: total diagonal population one, imaginary parts of the diagonal
  populations zero, u12 = conj(u21), all within 4 standard errors.
"""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import models, observables, sampling, shgb

PAR = dict(A=0.01, B=1.6, C=0.005, D=1.0, mass=2000.0)
EPS = 0.01


@pytest.fixture(scope="module")
def run():
    mdl = models.QCLE(**PAR)
    ens = sampling.init_beams(mdl, 600, EPS, 99, -2.5, 0.3, "normal", 30.0, 1.0, 1)
    ens0 = ens.subset(np.arange(ens.n))
    shgb.advance(mdl, ens, 700, 0.5, 99)
    return mdl, ens0, ens


def test_initial_state(run):
    mdl, ens0, _ = run
    c = observables.beam_integrals(ens0, EPS)
    np.testing.assert_allclose(c, 1.0, rtol=1e-14)
    assert (ens0.comp == 1).all()
    assert abs(ens0.X[:, 0].mean() + 2.5) < 4 * 0.3 / math.sqrt(600)
    assert abs(ens0.X[:, 1].std() - 1.0) < 0.1


def test_det_M_and_spd(run):
    _, _, ens = run
    np.testing.assert_allclose(np.linalg.det(ens.M), 1.0, atol=1e-9)
    assert (np.linalg.eigvalsh(ens.M) > 0).all()
    np.testing.assert_array_equal(ens.M, np.swapaxes(ens.M, 1, 2))


def test_weight_equals_twice_angle_change(run):
    mdl, ens0, ens = run
    assert (ens.X[:, 1] > 0).all()          # q1 monotone along every path
    th0 = mdl.mixing_angle(ens0.X[:, 0])
    th1 = mdl.mixing_angle(ens.X[:, 0])
    np.testing.assert_allclose(ens.logw + ens.Lam, 2 * np.abs(th1 - th0), rtol=1e-7, atol=1e-12)
    assert ens.nhop.mean() > 2.0            # most beams crossed: about pi hops each


def test_statistical_symmetries(run):
    _, _, ens = run
    n = ens.n
    sums = observables.populations(ens, EPS)
    mean, se = observables.population_mean_se(sums, n)
    assert abs(mean[0].real + mean[1].real - 1.0) < 4 * math.hypot(se[0].real, se[1].real)
    assert abs(mean[0].imag) < 4 * se[0].imag + 1e-12
    assert abs(mean[1].imag) < 4 * se[1].imag + 1e-12
    d = mean[3] - np.conj(mean[2])
    assert abs(d.real) < 4 * math.hypot(se[2].real, se[3].real)
    assert abs(d.imag) < 4 * math.hypot(se[2].imag, se[3].imag)


def test_trajectories_do_not_depend_on_eps(run):
    # the beam ODEs and the hop algorithm never read eps: only G does
    mdl, ens0, ens = run
    e = ens0.subset(np.arange(20))
    shgb.advance(mdl, e, 700, 0.5, 99)
    np.testing.assert_array_equal(e.X, ens.X[:20])
    np.testing.assert_array_equal(e.nhop, ens.nhop[:20])


def initial_law(sampling_mod, n=2000):
    """Sec. 2.5 sampling with q1 ~ N(-2.5, 0.3^2) and p1 ~ U[10, 30): (largest |beam integral - 1|,
    |mean q1 + 2.5| in standard errors, |std q1 - 0.3|, KS p-value of p1 against U[10, 30))."""
    mdl = models.QCLE(**PAR)
    ens = sampling_mod.init_beams(mdl, n, EPS, 7, -2.5, 0.3, "uniform", 10.0, 30.0, 1)
    c = observables.beam_integrals(ens, EPS)
    q, p = ens.X[:, 0], ens.X[:, 1]
    return (np.abs(c - 1.0).max(), abs(q.mean() + 2.5) / (0.3 / math.sqrt(n)), abs(q.std() - 0.3),
            stats.kstest((p - 10.0) / 20.0, "uniform").pvalue)


def test_initial_law_of_centres_and_amplitude():
    err_c, z_q, err_std, p_ks = initial_law(sampling)
    assert err_c < 1e-13 and z_q < 4.0 and err_std < 4 * 0.3 / math.sqrt(2 * 2000) and p_ks > 1e-3
