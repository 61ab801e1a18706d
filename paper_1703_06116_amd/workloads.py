"""Seeded synthetic inputs shaped like the paper's QCLE workloads.

Parameter tables and random draws only: no step of the method lives here.
Both the HIP path (bench, tests) and the CPU oracle (tests) receive their
inputs from this module; it imports neither.

Workloads (two-level QCLE, Sec. 3.3, with nuclear mass 2000):

* ``qcle1d_1e4``   1-D avoided crossing, 1e4 beams, 2000 RK4 steps of 0.5,
                   q ~ N(-5, 0.5^2), p ~ N(20, 1), lower surface, eps = 0.01.
* ``qcle1d_1e6``   same model, 1e6 beams, 4000 steps, p ~ U[10, 30];
                   populations and the field on a 64 x 64 grid of (q, p).
* ``qcle12d_2p18`` d = 12 nuclear coordinates (phase space m = 24): q2..q12
                   harmonic with w_k ~ U[0.002, 0.02] coupled to q1 by
                   lam = 1e-3, 2^18 beams, 2000 steps, eps = 0.02; the field at
                   16384 points scattered around beam centres.
* ``batch64_d12``  64 instances of the d = 12 model with C ~ U[0.002, 0.01],
                   eps from {0.01, 0.02, 0.05} and beam counts log-uniform in
                   [2^12, 2^17] (about 2.3e6 beams in all), 500 steps of 0.5,
                   FP32 trajectories with FP64 phase, one batched launch.
* ``qcle12d_grad`` the d = 12 model, 2^16 beams, 1000 steps, FP64: derivative of
                   the final upper-surface population in (A, B, C, D, p_mean).
"""

import numpy as np

POT = dict(A=0.01, B=1.6, C=0.005, D=1.0, mass=2000.0)

CONFIGS = {
    "qcle1d_1e4": dict(d=1, eps=0.01, n_beams=10_000, nsteps=2000, dt=0.5, q_mean=-5.0, q_std=0.5,
                       p_dist="normal", p_a=20.0, p_b=1.0, comp0=1, seed=0x1703061160000001,
                       n_points=0),
    "qcle1d_1e6": dict(d=1, eps=0.01, n_beams=1_000_000, nsteps=4000, dt=0.5, q_mean=-5.0, q_std=0.5,
                       p_dist="uniform", p_a=10.0, p_b=30.0, comp0=1, seed=0x1703061160000002,
                       n_points=4096),
    "qcle12d_2p18": dict(d=12, eps=0.02, n_beams=2**18, nsteps=2000, dt=0.5, q_mean=-5.0, q_std=0.5,
                         p_dist="normal", p_a=20.0, p_b=1.0, comp0=1, seed=0x1703061160000003,
                         n_points=16384, lam=1e-3),
    # pathwise derivative of the final upper-surface population in (A, B, C, D, p_mean)
    "qcle12d_grad": dict(d=12, eps=0.02, n_beams=2**16, nsteps=1000, dt=0.5, q_mean=-5.0, q_std=0.5,
                         p_dist="normal", p_a=20.0, p_b=1.0, comp0=1, seed=0x1703061160000005,
                         n_points=0, lam=1e-3),
}


# workloads whose bench step is the derivative of the populations
GRADIENT = ("qcle12d_grad",)

BATCH = {
    "batch64_d12": dict(n_inst=64, d=12, C=(0.002, 0.01), eps=(0.01, 0.02, 0.05), beams=(2**12, 2**17),
                        nsteps=500, dt=0.5, draw_seed=1703061164, seed0=0x1703061160000004),
}


def batch_instances(name, **overrides):
    """Per-instance configs of a batched workload (model parameters drawn once, seeded)."""
    b = dict(BATCH[name])
    b.update(overrides)
    rng = np.random.default_rng(b["draw_seed"])
    n = b["n_inst"]
    C = rng.uniform(*b["C"], n)
    eps = rng.choice(np.asarray(b["eps"]), n)
    lo, hi = np.log(b["beams"][0]), np.log(b["beams"][1])
    beams = np.exp(rng.uniform(lo, hi, n)).astype(np.int64)
    out = []
    for i in range(n):
        c = config("qcle12d_2p18", d=b["d"], bath_omega=bath_omega(b["d"]), C=float(C[i]), eps=float(eps[i]),
                   n_beams=int(beams[i]), nsteps=b["nsteps"], dt=b["dt"], seed=b["seed0"] + i, n_points=0)
        out.append(c)
    return out


def bath_omega(d, seed=1703061163):
    """Bath frequencies w_2..w_d ~ U[0.002, 0.02], drawn once."""
    if d <= 1:
        return np.zeros(0)
    return np.random.default_rng(seed).uniform(0.002, 0.02, d - 1)


def config(name, **overrides):
    c = dict(CONFIGS[name])
    c.update(POT)
    c.setdefault("lam", 0.0)
    c["bath_omega"] = bath_omega(c["d"])
    c.update(overrides)
    return c


def grid_points_2d(nq=64, npts=64, qlim=(0.0, 30.0), plim=(0.0, 35.0)):
    """Uniform (q, p) grid covering the final 1-D ensemble, row-major, (nq*npts, 2)."""
    q = np.linspace(qlim[0], qlim[1], nq)
    p = np.linspace(plim[0], plim[1], npts)
    Q, P = np.meshgrid(q, p, indexing="ij")
    return np.ascontiguousarray(np.stack([Q.ravel(), P.ravel()], 1))


def points_near(centres, eps, n, seed):
    """n points x = X_k + sqrt(eps) xi around randomly chosen centres."""
    rng = np.random.default_rng(seed)
    centres = np.asarray(centres, dtype=np.float64)
    k = rng.integers(0, centres.shape[0], n)
    return np.ascontiguousarray(centres[k] + np.sqrt(eps) * rng.normal(size=(n, centres.shape[1])))


def points_in_beams(centres, M, eps, n, seed):
    """n points drawn from the beams' own Gaussians: x = X_k + y, k a random beam, y ~ N(0, eps M_k^-1)
    (M_k the real part of beam k's Hessian), so that |G_k(x)| is about exp(-m/4) on average instead
    of vanishing in the beam's stiff directions."""
    rng = np.random.default_rng(seed)
    centres = np.asarray(centres, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    k = rng.integers(0, centres.shape[0], n)
    xi = rng.normal(size=(n, centres.shape[1]))
    L = np.linalg.cholesky(M[k])                                        # M = L L^T
    y = np.linalg.solve(np.swapaxes(L, 1, 2), xi[..., None])[..., 0]     # L^T y = xi: y ~ N(0, M^-1)
    return np.ascontiguousarray(centres[k] + np.sqrt(eps) * y)


def points_near_final(c, n, seed):
    """n evaluation points around a stand-in for the final ensemble of a QCLE workload.

    Centres: p1 from the workload's initial law, q1 = q0 + p1 T / M (free flight
    over T = nsteps dt), bath coordinates from their ground-state Wigner widths;
    each point is a centre plus sqrt(eps) times a standard normal vector.
    """
    rng = np.random.default_rng(seed)
    d, eps, M = c["d"], c["eps"], c["mass"]
    T = c["nsteps"] * c["dt"]
    X = np.zeros((n, 2 * d))
    if c["p_dist"] == "normal":
        p1 = rng.normal(c["p_a"], c["p_b"], n)
    else:
        p1 = rng.uniform(c["p_a"], c["p_b"], n)
    X[:, 0] = rng.normal(c["q_mean"], c["q_std"], n) + p1 * T / M
    X[:, d] = p1
    w = np.asarray(c["bath_omega"])
    if d > 1:
        X[:, 1:d] = rng.normal(size=(n, d - 1)) * np.sqrt(eps / (2 * M * w))
        X[:, d + 1:] = rng.normal(size=(n, d - 1)) * np.sqrt(eps * M * w / 2)
    return np.ascontiguousarray(X + np.sqrt(eps) * rng.normal(size=X.shape))


def synthetic_ensemble(n, m, seed, q_range=(5.0, 25.0), p_range=(10.0, 30.0), z_scale=0.5,
                       p_scale=1.0, s_scale=3.0, logw_scale=1.0, n_comp=4, a0=1.0):
    """A random beam state shaped like an evolved QCLE ensemble (host arrays).

    Centres spread over the ranges the ensemble reaches, Z = M + iN with M
    symmetric positive definite (M = I + L L^T / m) and N symmetric, phase
    space wave vectors P of size p_scale, phases S, weights exp(logw + Lam)
    with unit phase +-1, components uniform over n_comp.
    """
    rng = np.random.default_rng(seed)
    d = m // 2
    X = np.zeros((n, m))
    X[:, 0] = rng.uniform(*q_range, n)
    X[:, d] = rng.uniform(*p_range, n)
    if d > 1:
        X[:, 1:d] = rng.normal(0, 0.05, (n, d - 1))
        X[:, d + 1:] = rng.normal(0, 0.5, (n, d - 1))
    L = rng.normal(0, z_scale, (n, m, m))
    M = np.eye(m)[None] + L @ np.swapaxes(L, 1, 2) / m
    K = rng.normal(0, z_scale, (n, m, m))
    N = 0.5 * (K + np.swapaxes(K, 1, 2))
    return dict(
        X=X, P=rng.normal(0, p_scale, (n, m)), Z=M + 1j * N, S=rng.normal(0, s_scale, n),
        A=np.full(n, a0, dtype=np.complex128), logw=np.abs(rng.normal(0, logw_scale, n)),
        phase=rng.choice([-1.0, 1.0], n).astype(np.complex128), Lam=np.abs(rng.normal(0, 0.3, n)),
        E=rng.exponential(1.0, n), comp=rng.integers(0, n_comp, n), nhop=rng.integers(0, 5, n))
