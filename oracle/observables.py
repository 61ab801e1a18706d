"""Observables of the SHGB estimator (oracle), Sec. 2.3 eq:shgb and Sec. 2.4 steps 6-7.

    U_i(T, x) = E[ exp(omega(T)) G(T; x) delta_{i, l_T} ]
    G(x) = A exp( -(x-X)^T (M + iN) (x-X) / (2 eps) + i P.(x-X)/eps + i S/eps )   (Sec. 2, the beam G^eps)

with exp(omega) = exp(logw + Lam) * phase.

* ``beam_integrals``: the integral of exp(omega) G over x in R^m, by the
  Gaussian integral with Z = M + iN:
      (2 pi eps)^(m/2) det(Z)^(-1/2) exp(-P^T Z^-1 P / (2 eps)).
  The branch of det(Z)^(-1/2): Re Z = M is positive definite, so every
  eigenvalue of Z has a positive real part; det(Z)^(1/2) is the product of
  the principal square roots of the eigenvalues, the branch continuous from
  real Z.
* ``populations``: per component the sums over beams of c_k, Re c_k^2,
  Im c_k^2 and the count, from which mean and standard error follow; the
  population of component i is (1/N_traj) sum_{l_k = i} c_k.
* ``reconstruct``: the superposition at evaluation points, by a direct
  double sum over beams and points with y = x - X formed first.  Returns the
  unnormalised sum (divide by N_traj for U_i).
"""

import math

import numpy as np


def beam_weights(ens):
    """exp(omega) * A * exp(i S/eps) is applied by callers; this returns exp(omega) A."""
    return np.exp(ens.logw + ens.Lam) * ens.phase * ens.A


def beam_integrals(ens, eps):
    m = ens.m
    Z = ens.M + 1j * ens.N
    lam = np.linalg.eigvals(Z)                      # (n, m)
    sqrt_det = np.prod(np.sqrt(lam), axis=1)        # principal roots
    ZinvP = np.linalg.solve(Z, ens.P.astype(np.complex128)[..., None])[..., 0]
    quad = np.einsum("na,na->n", ens.P, ZinvP)
    gauss = (2.0 * math.pi * eps) ** (m / 2.0) / sqrt_det * np.exp(-quad / (2.0 * eps))
    return beam_weights(ens) * np.exp(1j * ens.S / eps) * gauss


def populations(ens, eps):
    """Array (n_comp, 5): [sum Re c, sum Im c, sum (Re c)^2, sum (Im c)^2, count]."""
    c = beam_integrals(ens, eps)
    out = np.zeros((ens.n_comp, 5))
    for i in range(ens.n_comp):
        sel = ens.comp == i
        ci = c[sel]
        out[i] = [ci.real.sum(), ci.imag.sum(), (ci.real**2).sum(), (ci.imag**2).sum(), sel.sum()]
    return out


def population_mean_se(sums, n_traj):
    """Mean and standard error of each component's population from the raw sums."""
    mean = (sums[:, 0] + 1j * sums[:, 1]) / n_traj
    var_re = sums[:, 2] / n_traj - mean.real**2
    var_im = sums[:, 3] / n_traj - mean.imag**2
    se = np.sqrt(np.maximum(var_re, 0.0) / max(n_traj - 1, 1)) + 1j * np.sqrt(
        np.maximum(var_im, 0.0) / max(n_traj - 1, 1))
    return mean, se


def reconstruct(ens, eps, points, chunk=4096):
    """Unnormalised sum_k exp(omega_k) G_k(x_q) per component: (n_comp, Q) complex."""
    points = np.asarray(points, dtype=np.float64)
    Q = points.shape[0]
    out = np.zeros((ens.n_comp, Q), dtype=np.complex128)
    w = beam_weights(ens) * np.exp(1j * ens.S / eps)
    Z = ens.M + 1j * ens.N
    for k0 in range(0, ens.n, chunk):
        sl = slice(k0, min(k0 + chunk, ens.n))
        y = points[None, :, :] - ens.X[sl, None, :]            # (k, Q, m)
        quad = np.einsum("kqa,kab,kqb->kq", y, Z[sl], y)
        lin = np.einsum("ka,kqa->kq", ens.P[sl], y)
        g = np.exp(-quad / (2.0 * eps) + 1j * lin / eps) * w[sl, None]
        for i in range(ens.n_comp):
            sel = ens.comp[sl] == i
            if sel.any():
                out[i] += g[sel].sum(0)
    return out


def reconstruct_abs(ens, eps, points, chunk=4096):
    """sum_k |exp(omega_k) G_k(x_q)| per component: the scale of each sum's rounding error."""
    points = np.asarray(points, dtype=np.float64)
    out = np.zeros((ens.n_comp, points.shape[0]))
    w = np.abs(beam_weights(ens))
    for k0 in range(0, ens.n, chunk):
        sl = slice(k0, min(k0 + chunk, ens.n))
        y = points[None, :, :] - ens.X[sl, None, :]
        quad = np.einsum("kqa,kab,kqb->kq", y, ens.M[sl], y)
        g = np.exp(-quad / (2.0 * eps)) * w[sl, None]
        for i in range(ens.n_comp):
            sel = ens.comp[sl] == i
            if sel.any():
                out[i] += g[sel].sum(0)
    return out
