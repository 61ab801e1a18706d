"""Pins for the oracle's populations and reconstruction (Sec. 2, the beam G^eps, Sec. 2.3 eq:shgb).

* the closed-form integral of a complex Gaussian beam against two-dimensional
  numerical quadrature (scipy dblquad), real and imaginary parts;
* a block-diagonal m = 4 beam against the product of pinned m = 2 integrals;
* the det(Z)^(-1/2) branch is continuous along Z(s) = M + i s N from real Z;
* the reconstructed field, integrated on a fine grid, equals the populations;
* the field of one beam has position expectation X and momentum expectation
  <-i eps grad> = P (derivative by FFT on a fine periodic grid): the beam is
  centred at X and carries the momentum P, which fixes the signs of x - X and
  of the linear phase term of the beam G^eps (Sec. 2).
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import observables, shgb


def random_beam(m, rng, eps):
    e = shgb.Ensemble(1, m, 4)
    e.X[0] = rng.normal(0, 1, m)
    e.P[0] = rng.normal(0, 0.6, m)
    L = rng.normal(0, 0.5, (m, m))
    e.M[0] = np.eye(m) * 0.7 + L @ L.T
    K = rng.normal(0, 0.8, (m, m))
    e.N[0] = 0.5 * (K + K.T)
    e.S[0] = rng.normal()
    e.A[0] = rng.normal() + 1j * rng.normal()
    e.logw[0] = rng.normal(0, 0.3)
    e.Lam[0] = abs(rng.normal(0, 0.3))
    e.phase[0] = -1.0
    return e


def beam_value(e, eps, x):
    y = x - e.X[0]
    Z = e.M[0] + 1j * e.N[0]
    w = math.exp(e.logw[0] + e.Lam[0]) * e.phase[0] * e.A[0]
    return w * np.exp(-y @ Z @ y / (2 * eps) + 1j * e.P[0] @ y / eps + 1j * e.S[0] / eps)


def dblquad_integral(e, eps):
    """The integral of the beam over the plane by two-dimensional quadrature."""
    L = 9.0 * math.sqrt(eps)
    x0, x1 = e.X[0]
    kw = dict(epsabs=1e-11, epsrel=1e-11)
    re, _ = integrate.dblquad(lambda b, a: beam_value(e, eps, np.array([a, b])).real,
                              x0 - L, x0 + L, x1 - L, x1 + L, **kw)
    im, _ = integrate.dblquad(lambda b, a: beam_value(e, eps, np.array([a, b])).imag,
                              x0 - L, x0 + L, x1 - L, x1 + L, **kw)
    return re + 1j * im


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_beam_integral_matches_dblquad(seed):
    rng = np.random.default_rng(seed)
    eps = 0.4
    e = random_beam(2, rng, eps)
    got = observables.beam_integrals(e, eps)[0]
    assert abs(got - dblquad_integral(e, eps)) < 1e-8 * max(1.0, abs(got))


def test_block_diagonal_beam_is_product_of_pinned_2d_integrals():
    rng = np.random.default_rng(7)
    eps = 0.3
    a, b = random_beam(2, rng, eps), random_beam(2, rng, eps)
    for e in (a, b):
        e.A[0] = 1.0
        e.S[0] = e.logw[0] = e.Lam[0] = 0.0
        e.phase[0] = 1.0
    big = shgb.Ensemble(1, 4, 4)
    big.X[0] = np.concatenate([a.X[0], b.X[0]])
    big.P[0] = np.concatenate([a.P[0], b.P[0]])
    big.M[0][:2, :2], big.M[0][2:, 2:] = a.M[0], b.M[0]
    big.N[0][:2, :2], big.N[0][2:, 2:] = a.N[0], b.N[0]
    big.A[0] = 1.0
    prod = observables.beam_integrals(a, eps)[0] * observables.beam_integrals(b, eps)[0]
    assert abs(observables.beam_integrals(big, eps)[0] - prod) < 1e-13 * abs(prod)


def test_sqrt_det_branch_is_continuous_from_real():
    rng = np.random.default_rng(11)
    m = 8
    L = rng.normal(0, 0.4, (m, m))
    M = np.eye(m) * 0.3 + L @ L.T
    K = rng.normal(0, 3.0, (m, m))
    N = 0.5 * (K + K.T)
    prev = None
    for s in np.linspace(0.0, 1.0, 4001):
        e = shgb.Ensemble(1, m, 1)
        e.M[0], e.N[0], e.A[0] = M, s * N, 1.0
        val = observables.beam_integrals(e, 1.0)[0]   # (2 pi)^(m/2) det(Z)^(-1/2)
        if prev is None:
            ref = (2 * math.pi) ** (m / 2) / math.sqrt(np.linalg.det(M))
            assert abs(val - ref) < 1e-12 * ref
        else:
            assert abs(val - prev) < 0.02 * abs(prev), s
        prev = val


def grid_integral_and_populations(obs):
    """The field of six beams summed over a fine grid, and the populations (module ``obs``)."""
    rng = np.random.default_rng(3)
    eps = 0.05
    ens = shgb.Ensemble(6, 2, 4)
    for k in range(6):
        b = random_beam(2, rng, eps)
        for f in ("X", "P", "M", "N", "S", "A", "logw", "Lam", "phase"):
            getattr(ens, f)[k] = getattr(b, f)[0]
    ens.X *= 0.3
    ens.comp[:] = [0, 1, 1, 2, 3, 3]
    pops = obs.populations(ens, eps)
    h = 0.01
    g = np.arange(-4.0, 4.0, h)
    pts = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    field = obs.reconstruct(ens, eps, pts)
    return field.sum(1) * h * h, pops


def test_reconstruction_integrates_to_population():
    integral, pops = grid_integral_and_populations(observables)
    np.testing.assert_allclose(integral.real, pops[:, 0], rtol=0, atol=1e-9 * np.abs(pops[:, :2]).max())
    np.testing.assert_allclose(integral.imag, pops[:, 1], rtol=0, atol=1e-9 * np.abs(pops[:, :2]).max())
    np.testing.assert_array_equal(pops[:, 4], [1, 2, 1, 2])


def field_moments(obs, eps=0.05, h=0.005, half=1.5):
    """Position and momentum expectations of one beam's field on a grid around its centre."""
    e = random_beam(2, np.random.default_rng(5), eps)
    e.comp[0] = 0
    g = np.arange(-half, half, h)
    gx, gy = np.meshgrid(e.X[0, 0] + g, e.X[0, 1] + g, indexing="ij")
    pts = np.stack([gx.ravel(), gy.ravel()], 1)
    u = obs.reconstruct(e, eps, pts)[0].reshape(gx.shape)
    rho = np.abs(u) ** 2
    x_mean = np.array([(gx * rho).sum(), (gy * rho).sum()]) / rho.sum()
    k = 2 * np.pi * np.fft.fftfreq(g.size, h)
    uh = np.fft.fft2(u)
    p_mean = []
    for ka in (k[:, None], k[None, :]):
        du = np.fft.ifft2(1j * ka * uh)
        p_mean.append((np.conj(u) * (-1j * eps) * du).sum().real / rho.sum())
    return e, x_mean, np.array(p_mean)


def test_field_is_centred_at_X_with_momentum_P():
    e, x_mean, p_mean = field_moments(observables)
    np.testing.assert_allclose(x_mean, e.X[0], rtol=0, atol=1e-9)
    np.testing.assert_allclose(p_mean, e.P[0], rtol=0, atol=1e-9)
    assert np.abs(e.P[0]).min() > 0.1
