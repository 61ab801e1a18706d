"""Initial beam parameters (oracle), Sec. 2.5 and Sec. 2.4 step 2.

Every beam starts as G(M0, N0, X0, P0, S0, A0; x) on one component with
omega = 0 and a fresh waiting-time threshold.  The beam shape is fixed
(reading of the workloads, which give only the distribution of centres):
M0 = identity, N0 = 0, P0 = 0, S0 = 0 and A0 = (2 pi eps)^(-m/2), so that
each beam integrates to one and the population at t = 0 is one on the
starting component.  Centres X0 = (q, p) in phase space:

* q1 ~ N(q_mean, q_std^2);
* p1 ~ N(p_a, p_b^2) (dist 'normal') or U[p_a, p_b) (dist 'uniform');
* bath modes k = 2..d: ground-state Wigner function of the harmonic mode
  with hbar replaced by eps, q_k ~ N(0, eps/(2 M w_k)), p_k ~ N(0, eps M w_k/2).

Normals come from the Box-Muller transform (Box & Muller 1958) applied to
Philox words; see ``oracle.philox`` for the counter layout.
"""

import math

import numpy as np

from . import philox
from .shgb import Ensemble, threshold


def normal(seed, gid, c):
    """Standard normal for phase-space coordinate c of beam gid."""
    w = philox.block(seed, gid, c // 4, philox.TAG_NORMAL)
    pair = (c % 4) // 2
    u1, u2 = philox.u01(w[2 * pair]), philox.u01(w[2 * pair + 1])
    r = math.sqrt(-2.0 * math.log(u1))
    return r * math.cos(2.0 * math.pi * u2) if c % 2 == 0 else r * math.sin(2.0 * math.pi * u2)


def uniform(seed, gid, c):
    return philox.u01(philox.block(seed, gid, c, philox.TAG_UNIF)[0])


def init_beams(model, n, eps, seed, q_mean, q_std, p_dist, p_a, p_b, comp0,
               beam_id_offset=0):
    """Sample n beams of the QCLE workloads (global ids beam_id_offset + 0..n-1)."""
    d, m = model.d, model.m
    ens = Ensemble(n, m, model.n_comp)
    for b in range(n):
        gid = beam_id_offset + b
        ens.gid[b] = gid
        x = np.zeros(m)
        x[0] = q_mean + q_std * normal(seed, gid, 0)
        if p_dist == "normal":
            x[d] = p_a + p_b * normal(seed, gid, d)
        elif p_dist == "uniform":
            x[d] = p_a + (p_b - p_a) * uniform(seed, gid, d)
        else:
            raise ValueError(p_dist)
        for k in range(1, d):
            w = model.bath_omega[k - 1]
            x[k] = math.sqrt(eps / (2.0 * model.mass * w)) * normal(seed, gid, k)
            x[d + k] = math.sqrt(eps * model.mass * w / 2.0) * normal(seed, gid, d + k)
        ens.X[b] = x
        ens.E[b] = threshold(philox.u01(philox.block(seed, gid, 0, philox.TAG_HOP)[1]))
    ens.M[:] = np.eye(m)
    ens.N[:] = 0.0
    ens.P[:] = 0.0
    ens.S[:] = 0.0
    ens.A[:] = (2.0 * math.pi * eps) ** (-m / 2.0)
    ens.logw[:] = 0.0
    ens.phase[:] = 1.0
    ens.Lam[:] = 0.0
    ens.comp[:] = comp0
    ens.nhop[:] = 0
    return ens
