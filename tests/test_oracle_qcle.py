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
from scipy import linalg, stats

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


def harmonic_ground_state(mass, w, eps, n=4001):
    """Ground state of H = -(eps^2 / 2 mass) d^2/dq^2 + mass w^2 q^2 / 2 (the bath mode with hbar
    replaced by eps), found by second-order finite differences on a uniform grid and
    scipy.linalg.eigh_tridiagonal: (energy, potential expectation, kinetic expectation, <q^2>)."""
    L = 12.0 * math.sqrt(eps / (mass * w))          # far beyond the classical turning points
    q = np.linspace(-L, L, n)
    h = q[1] - q[0]
    kin = eps**2 / (2.0 * mass * h * h)
    pot = 0.5 * mass * w * w * q * q
    lam, vec = linalg.eigh_tridiagonal(2.0 * kin + pot, np.full(n - 1, -kin), select="i", select_range=(0, 0))
    psi2 = vec[:, 0] ** 2
    V = float((pot * psi2).sum())
    return float(lam[0]), V, float(lam[0]) - V, float((q * q * psi2).sum())


def bath_law(sampling_mod, n=6000, seed=21):
    """Sec. 2.5 sampling of the d = 12 workload's bath modes (q_k, p_k), k = 2..12, against the
    ground state of each harmonic mode (the initial wave function of a bath in its ground state;
    its Wigner function is the phase-space law).  Per mode, in standard errors of the sample
    mean: total energy against the ground-state energy, potential and kinetic parts against the
    ground state's expectations; the q-p correlation in units of 1/sqrt(n); and the smaller KS
    p-value of q_k and p_k against the normal laws with the ground state's second moments.
    Returns the worst of each over the modes."""
    w = np.random.default_rng(1703061163).uniform(0.002, 0.02, 11)
    mdl = models.QCLE(**PAR, d=12, lam=1e-3, bath_omega=w)
    eps = 0.02
    ens = sampling_mod.init_beams(mdl, n, eps, seed, -5.0, 0.5, "normal", 20.0, 1.0, 1)
    worst = np.zeros(4)
    worst[3] = 1.0
    for k in range(1, 12):
        E0, V0, T0, q2 = harmonic_ground_state(mdl.mass, w[k - 1], eps)
        q, p = ens.X[:, k], ens.X[:, 12 + k]
        pot = 0.5 * mdl.mass * w[k - 1] ** 2 * q * q
        kin = p * p / (2.0 * mdl.mass)
        z = [abs(x.mean() - ref) / (x.std() / math.sqrt(n)) for x, ref in ((pot + kin, E0), (pot, V0), (kin, T0))]
        worst[0] = max(worst[0], z[0])
        worst[1] = max(worst[1], z[1], z[2])
        worst[2] = max(worst[2], abs(np.corrcoef(q, p)[0, 1]) * math.sqrt(n))
        p2 = 2.0 * mdl.mass * T0
        worst[3] = min(worst[3], stats.kstest(q / math.sqrt(q2), "norm").pvalue,
                       stats.kstest(p / math.sqrt(p2), "norm").pvalue)
    return worst


def test_harmonic_ground_state_solver_matches_zero_point_energy():
    # the solver itself: the lowest level of the oscillator is eps w / 2 (textbook), split evenly
    E0, V0, T0, _ = harmonic_ground_state(2000.0, 0.01, 0.02)
    assert abs(E0 - 0.5 * 0.02 * 0.01) < 1e-5 * E0 and abs(V0 - T0) < 1e-5 * E0


def test_bath_initial_law_is_the_ground_state_wigner_law():
    z_energy, z_parts, corr, p_ks = bath_law(sampling)
    assert z_energy < 4.0 and z_parts < 4.0 and corr < 4.0 and p_ks > 1e-3, (z_energy, z_parts, corr, p_ks)
