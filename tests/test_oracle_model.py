"""Pins for the oracle's QCLE coefficients (Sec. 3.3, eq:QCLE and the adiabatic quantities below it).

Independent references: numpy's symmetric eigensolver for the adiabatic
energies and the eigenvector angle, mpmath high-precision numerical
differentiation for derivatives up to third order, scipy quadrature for the
total coupling strength, and finite differences for every Jacobian/Hessian
the beam ODEs consume.
"""

import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import models

PAR = dict(A=0.01, B=1.6, C=0.005, D=1.0, mass=2000.0)


def qcle(d=1, mod=models):
    if d == 1:
        return mod.QCLE(**PAR)
    rng = np.random.default_rng(5)
    return mod.QCLE(**PAR, d=d, lam=1e-3, bath_omega=rng.uniform(0.002, 0.02, d - 1))


def vmat(mdl, r):
    """Diabatic 2x2 potential written from its definition."""
    q1 = r[0]
    vb = 0.0
    for k in range(1, mdl.d):
        vb += 0.5 * mdl.mass * mdl.bath_omega[k - 1] ** 2 * r[k] ** 2 + mdl.lam * q1 * r[k]
    a = mdl.A * math.tanh(mdl.B * q1)
    c = mdl.C * math.exp(-mdl.D * q1 * q1)
    return np.array([[a + vb, c], [c, -a + vb]])


def energy_errors(d, mod=models):
    """Energies of both surfaces against numpy.linalg.eigvalsh of the diabatic matrix."""
    mdl = qcle(d, mod)
    rng = np.random.default_rng(1)
    r = rng.normal(0, 1.5, size=(50, d))
    out = []
    for comp, pick in ((0, 1), (1, 0)):
        E = mdl.energy(r, np.full(50, comp))
        ref = np.array([np.linalg.eigvalsh(vmat(mdl, ri))[pick] for ri in r])
        out.append((E, ref))
    return out


@pytest.mark.parametrize("d", [1, 3])
def test_energies_match_eigvalsh(d):
    for E, ref in energy_errors(d):
        np.testing.assert_allclose(E, ref, rtol=1e-13, atol=1e-16)


def d21_and_angle_errors(mod=models):
    """Largest |d21 - d(angle)/dq| (relative to max(1, |fd|)) and |mixing angle - angle| on a grid."""
    # upper eigenvector (cos t, sin t) with t in (0, pi/2) because V12 > 0;
    # d21 = <phi2 | d phi1/dq> = dt/dq for phi2 = (-sin t, cos t)
    mdl = qcle(1, mod)
    h = 1e-5

    def angle(q):
        _, v = np.linalg.eigh(vmat(mdl, np.array([q])))
        up = v[:, 1] * np.sign(v[0, 1] + v[1, 1])
        return math.atan2(up[1], up[0])

    e_d21 = e_ang = 0.0
    for q in np.linspace(-3, 3, 25):
        fd = (angle(q + h) - angle(q - h)) / (2 * h)
        e_d21 = max(e_d21, abs(mdl.d21(np.array([q]))[0] - fd) / max(1.0, abs(fd)))
        e_ang = max(e_ang, abs(mdl.mixing_angle(np.array([q]))[0] - angle(q)))
    return e_d21, e_ang


def test_d21_is_derivative_of_eigenvector_angle():
    e_d21, e_ang = d21_and_angle_errors()
    assert e_d21 <= 1e-6 and e_ang < 1e-12


def test_s_derivatives_high_precision():
    mdl = qcle(1)
    mp.mp.dps = 40

    def s_mp(q):
        a = mp.mpf(mdl.A) * mp.tanh(mp.mpf(mdl.B) * q)
        c = mp.mpf(mdl.C) * mp.exp(-mp.mpf(mdl.D) * q * q)
        return mp.sqrt(a * a + c * c)

    for q in [-2.3, -0.7, -0.05, 0.0, 0.31, 1.2, 3.7]:
        for k in range(4):
            ref = float(mp.diff(s_mp, mp.mpf(q), k))
            got = mdl.s(np.array([q]), k)[0]
            assert abs(got - ref) <= 1e-11 * max(abs(ref), 1e-6), (q, k, got, ref)


def test_total_coupling_is_quarter_turn():
    # theta goes from pi/2 to 0 across the avoided crossing: int |d21| dq = pi/2
    mdl = qcle(1)
    val, err = integrate.quad(lambda q: abs(mdl.d21(np.array([q]))[0]), -40, 40,
                              points=[0.0], limit=400, epsabs=1e-13, epsrel=1e-13)
    assert abs(val - math.pi / 2) < 1e-9
    # d21 < 0 everywhere for these parameters and d21(0) = -A B / (2 C)
    q = np.linspace(-8, 8, 2001)
    assert (mdl.d21(q) < 0).all()
    assert abs(mdl.d21(np.array([0.0]))[0] + PAR["A"] * PAR["B"] / (2 * PAR["C"])) < 1e-12


def _fd_jac(f, x, h):
    cols = []
    for b in range(x.size):
        e = np.zeros_like(x)
        e[b] = h
        cols.append((f(x + e) - f(x - e)) / (2 * h))
    return np.stack(cols, axis=-1)


@pytest.mark.parametrize("d", [1, 3])
@pytest.mark.parametrize("comp", [0, 1, 2, 3])
def test_jacobians_and_hessians_by_finite_differences(d, comp):
    mdl = qcle(d)
    m = 2 * d
    rng = np.random.default_rng(comp + 10 * d)
    for _ in range(5):
        x = np.concatenate([rng.normal(0, 1.0, d), rng.normal(15, 3, d)])
        P = rng.normal(0, 1, m)
        c1 = np.array([comp])
        J = mdl.jac_alpha(x[None], c1)[0]
        Jfd = _fd_jac(lambda z: mdl.alpha(z[None], c1)[0], x, 1e-5)
        np.testing.assert_allclose(J, Jfd, atol=1e-9)
        g = mdl.grad_beta(x[None], c1)[0]
        gfd = _fd_jac(lambda z: mdl.beta(z[None], c1), x, 1e-6)[0]
        np.testing.assert_allclose(g, gfd, atol=1e-9)
        H = mdl.hess_beta(x[None], c1)[0]
        Hfd = _fd_jac(lambda z: mdl.grad_beta(z[None], c1)[0], x, 1e-5)
        np.testing.assert_allclose(H, Hfd, atol=1e-8)
        HP = mdl.hess_P_alpha(x[None], c1, P[None])[0]

        def grad_Palpha(z):
            return (P @ mdl.jac_alpha(z[None], c1)[0])   # d/dx_b (P . alpha)
        HPfd = _fd_jac(grad_Palpha, x, 1e-5)
        np.testing.assert_allclose(HP, HPfd, atol=1e-8)


@pytest.mark.parametrize("d", [1, 3])
def test_energy_gradient_matches_eigvalsh_differences(d):
    mdl = qcle(d)
    rng = np.random.default_rng(3)
    for _ in range(5):
        r = rng.normal(0, 1.0, d)
        for comp, pick in ((0, 1), (1, 0)):
            g = mdl.grad_energy(r[None], np.array([comp]))[0]
            gfd = _fd_jac(lambda z: np.array([np.linalg.eigvalsh(vmat(mdl, z))[pick]]), r, 1e-6)[0]
            np.testing.assert_allclose(g, gfd, atol=1e-9)


def test_coupling_structure_conserves_trace():
    # d/dt (int u11 + int u22): the gamma terms of rows 0 and 1 cancel for every source
    mdl = qcle(1)
    X = np.array([[0.3, 20.0], [-1.0, 11.0]])
    G = mdl.gamma(X)
    np.testing.assert_array_equal(G[:, 0, :] + G[:, 1, :], 0.0)
    # every component leaves at total rate 2|kappa| towards two equally likely targets
    for l in range(4):
        col = np.abs(G[:, :, l])
        np.testing.assert_allclose(col.sum(1), 2 * np.abs(mdl.kappa(X)))
        assert (np.count_nonzero(col, axis=1) == 2).all()
    # u12 = conj(u21): rows 2 and 3 are conjugate (real gamma: equal), betas opposite
    np.testing.assert_array_equal(G[:, 2, :2], G[:, 3, :2])
    comp2, comp3 = np.array([2, 2]), np.array([3, 3])
    np.testing.assert_array_equal(mdl.beta(X, comp2), -mdl.beta(X, comp3))


@pytest.mark.parametrize("comp", [0, 1])
def test_paper32_derivatives_by_finite_differences(comp):
    """Eq:ex2: every Jacobian/Hessian the beam ODEs use equals central differences."""
    mdl = models.Paper32()
    rng = np.random.default_rng(40 + comp)
    for _ in range(6):
        x = rng.normal(0, 1.2, 2)
        P = rng.normal(0, 1, 2)
        c1 = np.array([comp])
        np.testing.assert_allclose(mdl.jac_alpha(x[None], c1)[0],
                                   _fd_jac(lambda z: mdl.alpha(z[None], c1)[0], x, 1e-5), atol=1e-9)
        np.testing.assert_allclose(mdl.grad_beta(x[None], c1)[0],
                                   _fd_jac(lambda z: mdl.beta(z[None], c1), x, 1e-6)[0], atol=1e-8)
        np.testing.assert_allclose(mdl.hess_beta(x[None], c1)[0],
                                   _fd_jac(lambda z: mdl.grad_beta(z[None], c1)[0], x, 1e-5), atol=1e-8)
        np.testing.assert_allclose(mdl.hess_P_alpha(x[None], c1, P[None])[0],
                                   _fd_jac(lambda z: P @ mdl.jac_alpha(z[None], c1)[0], x, 1e-5), atol=1e-8)


def test_paper32_coefficients_as_printed():
    """Spot values read off eq:ex2 at a point, component by component."""
    mdl = models.Paper32()
    x = np.array([[0.3, -0.7]])
    r2 = 0.3 ** 2 + 0.7 ** 2
    np.testing.assert_allclose(mdl.alpha(x, np.array([0]))[0], [-np.sin(-0.4), -np.cos(1.0)])
    np.testing.assert_allclose(mdl.alpha(x, np.array([1]))[0], [-np.sin(1.0), -np.cos(-0.4)])
    assert mdl.beta(x, np.array([0]))[0] == np.sin(r2) and mdl.beta(x, np.array([1]))[0] == np.cos(r2)
    G = mdl.gamma(x)[0]
    np.testing.assert_allclose(G, r2 * np.array([[-1, 5], [-5, -0.5]]))
