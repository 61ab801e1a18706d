"""Pins for the oracle's beam ODEs, RK4 and Gaussian superposition.

P1  linear alpha, quadratic beta, constant gamma (Sec. 3.1 class): the beam
    ODEs are linear with constant coefficients and X, P, M, N, A have closed
    forms by matrix exponentials (scipy.linalg.expm); S by quadrature.
P2  same class: the Gaussian beam is the exact solution of the transport
    equation, which is also u(T, x) = u0(x(0)) exp(int (i beta/eps + gamma))
    along the characteristic through x (solve_ivp backwards).
P2b nonlinear scalar transport (pendulum flow, beta = 0) with an oscillating
    initial beam: the beam approximates the exact solution with an error that
    shrinks as eps -> 0; a wrong curvature term Hess(P.alpha) would leave an
    O(1) error.
"""

import math

import numpy as np
import pytest
from scipy import integrate, linalg

from oracle import models, observables, shgb


def random_linquad(m, seed, n=1):
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 0.5, (n, m))
    J = rng.normal(0, 0.4, (n, m, m))
    b0 = rng.normal(0, 1, n)
    b = rng.normal(0, 0.5, (n, m))
    H = rng.normal(0, 0.5, (n, m, m))
    H = 0.5 * (H + np.swapaxes(H, 1, 2))
    G = np.diag(rng.normal(-0.3, 0.2, n) + 1j * rng.normal(0, 0.3, n))
    return models.LinQuad(a, J, b0, b, H, G)


def one_beam(m, seed):
    rng = np.random.default_rng(seed + 100)
    ens = shgb.Ensemble(1, m, 1)
    ens.X[0] = rng.normal(0, 1, m)
    ens.P[0] = rng.normal(0, 1, m)
    Lm = rng.normal(0, 0.3, (m, m))
    ens.M[0] = np.eye(m) + Lm @ Lm.T
    Nm = rng.normal(0, 0.3, (m, m))
    ens.N[0] = 0.5 * (Nm + Nm.T)
    ens.S[0] = rng.normal()
    ens.A[0] = 0.7 - 0.2j
    ens.E[0] = np.inf          # gamma is diagonal: no hops
    return ens


def exact_beam(model, ens, T):
    m = model.m
    a, J, b, H, b0 = model.a[0], model.J[0], model.b[0], model.H[0], model.b0[0]
    # (X, P, 1)' = [[J, 0, a], [H, -J^T, b], [0, 0, 0]] (X, P, 1)
    K = np.zeros((2 * m + 1, 2 * m + 1))
    K[:m, :m] = J
    K[:m, -1] = a
    K[m:2 * m, :m] = H
    K[m:2 * m, m:2 * m] = -J.T
    K[m:2 * m, -1] = b
    v0 = np.concatenate([ens.X[0], ens.P[0], [1.0]])
    vT = linalg.expm(K * T) @ v0
    XT, PT = vT[:m], vT[m:2 * m]

    def X_at(t):
        return (linalg.expm(K * t) @ v0)[:m]

    S_int, _ = integrate.quad(lambda t: b0 + b @ X_at(t) + 0.5 * X_at(t) @ H @ X_at(t), 0, T,
                              epsabs=1e-13, epsrel=1e-13, limit=200)
    # vec(Z)' = L vec(Z) - i vec(H),  L Z = -Z J - J^T Z
    L = np.zeros((m * m, m * m))
    for k in range(m * m):
        E = np.zeros(m * m)
        E[k] = 1.0
        Em = E.reshape(m, m)
        L[:, k] = (-Em @ J - J.T @ Em).ravel()
    KZ = np.zeros((m * m + 1, m * m + 1), dtype=np.complex128)
    KZ[:m * m, :m * m] = L
    KZ[:m * m, -1] = -1j * H.ravel()
    z0 = np.concatenate([(ens.M[0] + 1j * ens.N[0]).ravel(), [1.0]])
    ZT = (linalg.expm(KZ * T) @ z0)[:m * m].reshape(m, m)
    AT = ens.A[0] * np.exp(model.G[0, 0] * T)
    return XT, PT, ZT, ens.S[0] + S_int, AT


def run_rk4(model, ens, T, nsteps, scheme="rk4"):
    e = ens.subset([0])
    for _ in range(nsteps):
        shgb.advance_interval(model, e, T / nsteps, seed=1, scheme=scheme)
    return e


@pytest.mark.parametrize("m", [2, 4])
def test_P1_exact_propagation_and_order4(m):
    model = random_linquad(m, seed=m)
    ens = one_beam(m, seed=m)
    T = 1.5
    XT, PT, ZT, ST, AT = exact_beam(model, ens, T)
    errs = []
    for n in (20, 40, 80):
        e = run_rk4(model, ens, T, n)
        err = max(np.abs(e.X[0] - XT).max(), np.abs(e.P[0] - PT).max(),
                  np.abs(e.M[0] + 1j * e.N[0] - ZT).max(), abs(e.S[0] - ST), abs(e.A[0] - AT))
        errs.append(err)
    assert errs[-1] < 1e-6
    for e1, e2 in zip(errs, errs[1:]):
        assert 12.0 < e1 / e2 < 20.0, errs          # fourth order: ratio 16
    e = run_rk4(model, ens, T, 640)
    np.testing.assert_allclose(e.X[0], XT, rtol=0, atol=1e-11)
    np.testing.assert_allclose(e.M[0] + 1j * e.N[0], ZT, rtol=0, atol=1e-11 * np.abs(ZT).max())
    assert abs(e.S[0] - ST) < 1e-10 and abs(e.A[0] - AT) < 1e-11


@pytest.mark.parametrize("m", [2, 4])
def test_P1_exact_propagation_and_order3(m):
    """Kutta's third-order scheme against the same closed form: error ratio 8 on halving."""
    model = random_linquad(m, seed=m)
    ens = one_beam(m, seed=m)
    T = 1.5
    XT, PT, ZT, ST, AT = exact_beam(model, ens, T)
    errs = []
    for n in (40, 80, 160):
        e = run_rk4(model, ens, T, n, scheme="rk3")
        errs.append(max(np.abs(e.X[0] - XT).max(), np.abs(e.P[0] - PT).max(),
                        np.abs(e.M[0] + 1j * e.N[0] - ZT).max(), abs(e.S[0] - ST), abs(e.A[0] - AT)))
    assert errs[-1] < 1e-4
    for e1, e2 in zip(errs, errs[1:]):
        assert 6.5 < e1 / e2 < 9.5, errs            # third order: ratio 8


def exact_field(model, ens0, eps, T, x):
    """u(T, x) for the scalar linear-quadratic system from its characteristic."""
    a, J, b, H, b0 = model.a[0], model.J[0], model.b[0], model.H[0], model.b0[0]
    m = model.m

    def f(t, z):
        xx = z[:m]
        return np.concatenate([a + J @ xx, [b0 + b @ xx + 0.5 * xx @ H @ xx]])

    sol = integrate.solve_ivp(f, (T, 0.0), np.concatenate([x, [0.0]]), method="DOP853",
                              rtol=1e-13, atol=1e-13)
    x0 = sol.y[:m, -1]
    phase_int = -sol.y[m, -1]          # int_0^T beta(x(s)) ds
    y = x0 - ens0.X[0]
    Z0 = ens0.M[0] + 1j * ens0.N[0]
    g0 = ens0.A[0] * np.exp(-y @ Z0 @ y / (2 * eps) + 1j * ens0.P[0] @ y / eps + 1j * ens0.S[0] / eps)
    return g0 * np.exp(1j * phase_int / eps + model.G[0, 0] * T)


@pytest.mark.parametrize("m", [2, 3])
def test_P2_beam_is_exact_pde_solution(m):
    model = random_linquad(m, seed=10 + m)
    ens = one_beam(m, seed=10 + m)
    eps, T = 0.3, 1.0
    e = run_rk4(model, ens, T, 400)
    rng = np.random.default_rng(4)
    pts = e.X[0] + rng.normal(0, 0.8, (12, m))
    got = observables.reconstruct(e, eps, pts)[0]
    ref = np.array([exact_field(model, ens, eps, T, x) for x in pts])
    scale = np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-9 * scale)


class Pendulum:
    """Scalar transport with alpha = (p, -sin q), beta = 0, gamma = 0 (test fixture)."""
    n_comp, m = 1, 2

    def alpha(self, X, comp):
        return np.stack([X[:, 1], -np.sin(X[:, 0])], 1)

    def jac_alpha(self, X, comp):
        J = np.zeros((X.shape[0], 2, 2))
        J[:, 0, 1] = 1.0
        J[:, 1, 0] = -np.cos(X[:, 0])
        return J

    def beta(self, X, comp):
        return np.zeros(X.shape[0])

    def grad_beta(self, X, comp):
        return np.zeros_like(X)

    def hess_beta(self, X, comp):
        return np.zeros((X.shape[0], 2, 2))

    def hess_P_alpha(self, X, comp, P):
        H = np.zeros((X.shape[0], 2, 2))
        H[:, 0, 0] = P[:, 1] * np.sin(X[:, 0])      # d^2/dq^2 of -P_p sin q
        return H

    def gamma(self, X):
        return np.zeros((X.shape[0], 1, 1), dtype=np.complex128)


def _pendulum_error(eps, hess_sign=1.0):
    model = Pendulum()
    if hess_sign != 1.0:
        base = model.hess_P_alpha
        model.hess_P_alpha = lambda X, c, P: hess_sign * base(X, c, P)
    ens = shgb.Ensemble(1, 2, 1)
    ens.X[0] = [0.4, 0.9]
    ens.P[0] = [0.8, -0.6]
    ens.M[0] = np.eye(2)
    ens.A[0] = 1.0
    ens.E[0] = np.inf
    T = 1.2
    e = ens.subset([0])
    for _ in range(240):
        shgb.advance_interval(model, e, T / 240, seed=0)

    def back(t, z):
        return [z[1], -math.sin(z[0])]

    rng = np.random.default_rng(0)
    pts = e.X[0] + math.sqrt(eps) * rng.normal(0, 1.0, (16, 2))
    got = observables.reconstruct(e, eps, pts)[0]
    ref = []
    for x in pts:
        sol = integrate.solve_ivp(back, (T, 0), x, method="DOP853", rtol=1e-12, atol=1e-12)
        y = sol.y[:, -1] - ens.X[0]
        ref.append(np.exp(-y @ y / (2 * eps) + 1j * ens.P[0] @ y / eps))
    ref = np.array(ref)
    return np.abs(got - ref).max()


def test_P2b_nonlinear_error_vanishes_with_eps():
    errs = [_pendulum_error(eps) for eps in (1e-2, 1e-3, 1e-4)]
    assert errs[2] < errs[0] / 5.0, errs
    assert errs[2] < 0.05, errs
    # the curvature term of the phase matters: flipping it leaves an O(1) error
    bad = _pendulum_error(1e-4, hess_sign=-1.0)
    assert bad > 10 * errs[2], (bad, errs)
