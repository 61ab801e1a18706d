"""GPU path for linear-quadratic systems (m = 2): the exact-solution pins on
the GPU and parity with the oracle.

* P1 on the GPU: linear alpha, quadratic beta, diagonal gamma -- the beam
  ODEs have closed forms (matrix exponentials); the GPU's RK4 converges to
  them at fourth order and agrees with the oracle to 1e-10.
* The system of Sec. 3.1 (eq:ex1): two components, dense J, gamma with a
  nonzero diagonal; GPU init + stepping against the oracle, hop sequences
  bit-exact apart from oracle-reported ties.
* P3 on the GPU: x-independent coefficients with complex gamma; the mean
  populations of a large GPU ensemble match the matrix exponential of
  Sec. 2.2 within their standard error.
"""

import math

import numpy as np
import pytest
import torch
from scipy import linalg

from oracle import models, observables, philox, shgb as oshgb

from _parity import arrays_from_ensemble, compare_states, ensemble_from_arrays
from test_oracle_gb import exact_beam, random_linquad
from test_oracle_hopping import B0, EPS, GAM

pytestmark = pytest.mark.gpu


def gpu_lq(gpu, model, eps):
    return gpu.make_linquad_model(eps, model.a, model.J, model.b0, model.b, model.H, model.G)


def random_beams(m, n, seed, n_comp=1, comp=0):
    """Beams with random centres, wave vectors, SPD Re Z, phases and amplitudes (host arrays)."""
    rng = np.random.default_rng(seed)
    e = oshgb.Ensemble(n, m, n_comp)
    e.gid[:] = np.arange(n, dtype=np.uint64)
    e.X[:] = rng.normal(0, 1, (n, m))
    e.P[:] = rng.normal(0, 1, (n, m))
    L = rng.normal(0, 0.3, (n, m, m))
    e.M[:] = np.eye(m) + L @ np.swapaxes(L, 1, 2)
    K = rng.normal(0, 0.3, (n, m, m))
    e.N[:] = 0.5 * (K + np.swapaxes(K, 1, 2))
    e.S[:] = rng.normal(0, 1, n)
    e.A[:] = rng.normal(0, 1, n) + 1j * rng.normal(0, 1, n)
    e.comp[:] = comp
    for b in range(n):
        e.E[b] = oshgb.threshold(philox.u01(philox.block(seed, b, 0, philox.TAG_HOP)[1]))
    return e


def test_P1_gpu_converges_to_exact_beam_at_order_4(gpu):
    model = random_linquad(2, seed=2)
    e0 = random_beams(2, 37, seed=7)
    e0.E[:] = 1e300                       # gamma is diagonal: no hops
    T = 1.5
    exact = [exact_beam(model, e0.subset([b]), T) for b in range(e0.n)]
    mdl = gpu_lq(gpu, model, eps=0.1)
    errs = []
    for n in (20, 40, 80, 640):
        st = gpu.pack(arrays_from_ensemble(e0))
        gpu.step_ensemble(mdl, st, n, T / n, 1)
        g = gpu.unpack(st)
        err = 0.0
        for b, (XT, PT, ZT, ST, AT) in enumerate(exact):
            err = max(err, np.abs(g["X"][b] - XT).max(), np.abs(g["P"][b] - PT).max(),
                      np.abs(g["Z"][b] - ZT).max(), abs(g["S"][b] - ST), abs(g["A"][b] - AT))
        errs.append(err)
    for e1, e2 in zip(errs[:2], errs[1:3]):
        assert 12.0 < e1 / e2 < 20.0, errs        # fourth order: ratio 16
    assert errs[3] < 1e-10, errs


def test_P1_gpu_matches_oracle(gpu):
    model = random_linquad(2, seed=5)
    e0 = random_beams(2, 3 * 256 + 11, seed=3)
    e0.E[:] = 1e300
    st = gpu.pack(arrays_from_ensemble(e0))
    gpu.step_ensemble(gpu_lq(gpu, model, 0.1), st, 60, 0.025, 1)
    e = e0.subset(np.arange(e0.n))
    oshgb.advance(model, e, 60, 0.025, 1)
    compare_states(gpu.unpack(st), e, label="P1")


def paper_system_31():
    """Eq:ex1 written as d_t u + alpha.grad u = (i/eps) beta u + gamma u (second
    equation's x2-derivative acting on u2)."""
    a = [[-1.0, 1.0], [1.0, -1.0]]
    J = [[[-1.0, -1.0], [-2.0, 1.0]], [[-0.5, -1.0], [-1.0, 0.5]]]
    b0 = [0.0, 0.0]
    b = [[0.0, 0.0], [0.0, 0.0]]
    H = [[[2.0, 0.0], [0.0, 2.0]], [[2.0, 2.0], [2.0, 2.0]]]
    G = [[-1.0, 0.5], [2.0 / 3.0, -2.0]]
    return models.LinQuad(a, J, b0, b, H, G)


@pytest.mark.parametrize("n,nsteps,dt", [(2 * 256 + 29, 50, 0.01), (300, 25, 0.04)])
def test_paper_system_31_gpu_matches_oracle(gpu, n, nsteps, dt):
    eps, seed = 0.1, 0x5EC31
    model = paper_system_31()
    mdl = gpu_lq(gpu, model, eps)
    sd = math.sqrt(1.0 - eps)       # centres from the normal law of Sec. 3.1, A0 = 1/eps
    st = gpu.State(n, 2)
    gpu.init_beams(mdl, gpu.make_init_spec(0.0, sd, "normal", 0.0, sd, 0, a0=1.0 / eps), st, seed)
    e0 = ensemble_from_arrays(gpu_init_reference(n, eps, seed, sd), n_comp=2)
    g0 = gpu.unpack(st)
    assert np.abs(g0["X"] - e0.X).max() <= 1e-13 * np.abs(e0.X).max()
    np.testing.assert_array_equal(g0["A"], e0.A)
    diag = gpu.new_diag()
    gpu.step_ensemble(mdl, st, nsteps, dt, seed, diag)
    e = e0.subset(np.arange(n))
    oshgb.advance(model, e, nsteps, dt, seed)
    errs, ties = compare_states(gpu.unpack(st), e, label="eq:ex1")
    d = diag.cpu().numpy()
    assert d[0] == e.nhop.sum() and e.nhop.sum() > n // 10
    pops = gpu.populations(mdl, st).cpu().numpy()
    ref = observables.populations(e, eps)
    ci = observables.beam_integrals(e, eps)
    assert np.abs(pops[:2, :2] - ref[:2, :2]).max() <= 1e-10 * np.abs(ci).sum()
    print("eq:ex1", errs, "ties", ties, "hops", int(d[0]))


def gpu_init_reference(n, eps, seed, sd):
    """The oracle's sampler for the centres of Sec. 3.1 (normal in both coordinates)."""
    from oracle import sampling
    X = np.zeros((n, 2))
    E = np.zeros(n)
    for b in range(n):
        X[b, 0] = sd * sampling.normal(seed, b, 0)
        X[b, 1] = sd * sampling.normal(seed, b, 1)
        E[b] = oshgb.threshold(philox.u01(philox.block(seed, b, 0, philox.TAG_HOP)[1]))
    return dict(X=X, P=np.zeros((n, 2)), Z=np.broadcast_to(np.eye(2), (n, 2, 2)).astype(np.complex128),
                S=np.zeros(n), A=np.full(n, 1.0 / eps, dtype=np.complex128), logw=np.zeros(n),
                phase=np.ones(n, dtype=np.complex128), Lam=np.zeros(n), E=E, comp=np.zeros(n, dtype=np.int64),
                nhop=np.zeros(n, dtype=np.int64))


def test_P3_gpu_populations_match_matrix_exponential(gpu):
    model = models.LinQuad.xindep(B0, GAM)
    mdl = gpu_lq(gpu, model, EPS)
    n, T, steps, seed = 200_000, 1.0, 10, 17
    st = gpu.State(n, 2)
    gpu.init_beams(mdl, gpu.make_init_spec(0.0, 0.0, "normal", 0.0, 0.0, 0), st, seed)
    gpu.step_ensemble(mdl, st, steps, T / steps, seed)
    mean, se = gpu.population_mean_se(gpu.populations(mdl, st).cpu().numpy(), n)
    exact = linalg.expm(T * (1j * np.diag(B0) / EPS + GAM))[:, 0]
    for i in range(3):
        assert abs(mean[i].real - exact[i].real) < 4 * se[i].real + 1e-4, (i, mean, exact, se)
        assert abs(mean[i].imag - exact[i].imag) < 4 * se[i].imag + 1e-4, (i, mean, exact, se)
    assert np.abs(exact).min() > 0.05 and se.real.max() < 0.01


def test_hop_entry_point_complex_gamma(gpu):
    model = models.LinQuad.xindep(B0, GAM)
    e0 = random_beams(2, 200, seed=9, n_comp=3)
    e0.comp[:] = np.arange(200) % 3
    e0.Lam[:] = np.linspace(0.0, 1.0, 200)
    e0.nhop[:] = np.arange(200) % 5
    st = gpu.pack(arrays_from_ensemble(e0))
    idx = np.arange(0, 200, 2, dtype=np.int32)
    gpu.hop(gpu_lq(gpu, model, EPS), st, torch.from_numpy(idx).cuda(), 5)
    g = gpu.unpack(st)
    e = e0.subset(np.arange(200))
    oshgb.hop_event(model, e, idx, 5)
    ok = e.dest_ties == 0
    np.testing.assert_array_equal(g["comp"][ok], e.comp[ok])
    np.testing.assert_array_equal(g["nhop"], e.nhop)
    assert np.abs(g["phase"] - e.phase).max() < 1e-15
    assert np.abs(g["logw"] - e.logw).max() < 1e-15 and (g["Lam"][idx] == 0).all()
    np.testing.assert_allclose(g["E"], e.E, rtol=1e-14)


# ---------------------------------------------------------------------------
# The nonlinear system of Sec. 3.2, eq:ex2: x-dependent transport, phases
# and couplings; beam curvature terms Hess(P.alpha) and Hess(beta) nonzero.

def test_paper_system_32_gpu_matches_oracle(gpu):
    model = models.Paper32()
    e0 = random_beams(2, 2 * 256 + 19, seed=21, n_comp=2)
    e0.X[:] *= 0.8
    e0.comp[:] = np.arange(e0.n) % 2
    e0.A[:] = 1.0
    st = gpu.pack(arrays_from_ensemble(e0))
    diag = gpu.new_diag()
    gpu.step_ensemble(gpu.make_paper32_model(0.04), st, 80, 0.01, 21, diag)
    e = e0.subset(np.arange(e0.n))
    oshgb.advance(model, e, 80, 0.01, 21)
    errs, ties = compare_states(gpu.unpack(st), e, label="eq:ex2")
    assert diag.cpu().numpy()[0] == e.nhop.sum() and e.nhop.sum() > e0.n // 4
    print("eq:ex2", errs, "ties", ties, "hops", e.nhop.sum())


def test_paper_system_32_from_the_single_initial_beam(gpu):
    """u1(0, x) = exp(-|x|^2/(2 eps)): every trajectory starts as the same beam (X = 0, Z = I,
    A = 1); only the hop times differ.  GPU init + stepping + populations against the oracle."""
    eps, n, nsteps, dt, seed = 0.02, 3 * 256 + 7, 100, 0.005, 0x5EC32
    mdl = gpu.make_paper32_model(eps)
    st = gpu.State(n, 2)
    gpu.init_beams(mdl, gpu.make_init_spec(0.0, 0.0, "normal", 0.0, 0.0, 0, a0=1.0), st, seed)
    a = gpu_init_reference(n, eps, seed, 0.0)
    a["A"] = np.ones(n, dtype=np.complex128)
    e0 = ensemble_from_arrays(a, n_comp=2)
    g0 = gpu.unpack(st)
    assert (g0["X"] == 0).all() and (g0["A"] == 1).all()
    np.testing.assert_allclose(g0["E"], e0.E, rtol=1e-14)
    gpu.step_ensemble(mdl, st, nsteps, dt, seed)
    e = e0.subset(np.arange(n))
    oshgb.advance(models.Paper32(), e, nsteps, dt, seed)
    compare_states(gpu.unpack(st), e, label="eq:ex2 single beam")
    pops = gpu.populations(mdl, st).cpu().numpy()
    ref = observables.populations(e, eps)
    ci = observables.beam_integrals(e, eps)
    assert np.abs(pops[:2, :2] - ref[:2, :2]).max() <= 1e-10 * np.abs(ci).sum()
    assert e.nhop.sum() > 0


def test_hop_entry_point_paper_system_32(gpu):
    model = models.Paper32()
    e0 = random_beams(2, 150, seed=23, n_comp=2)
    e0.comp[:] = np.arange(150) % 2
    e0.Lam[:] = np.linspace(0.0, 2.0, 150)
    e0.X[0] = 0.0                      # no coupling at the origin: counted, no hop
    st = gpu.pack(arrays_from_ensemble(e0))
    idx = np.arange(0, 150, 3, dtype=np.int32)
    diag = gpu.new_diag()
    gpu.hop(gpu.make_paper32_model(0.05), st, torch.from_numpy(idx).cuda(), 8, diag)
    g = gpu.unpack(st)
    e = e0.subset(np.arange(150))
    oshgb.hop_event(model, e, idx, 8)
    np.testing.assert_array_equal(g["comp"], e.comp)
    np.testing.assert_array_equal(g["nhop"], e.nhop)
    np.testing.assert_array_equal(g["phase"], e.phase)
    assert np.abs(g["logw"] - e.logw).max() < 1e-15
    assert diag.cpu().numpy()[6] == 1 == e.zero_rate.sum()


def test_paper_31_field_error_falls_as_inverse_square_root(gpu):
    """The convergence study of Sec. 3.1 in kind: for eq:ex1 the expectation of
    the method is the exact solution (the O(eps^(1/2)) residuals vanish), so the
    L2 distance between an N-trajectory field and the field of 2^22 trajectories
    (standing in for the N -> infinity limit, the paper's finite-volume reference
    being out of scope) is Monte Carlo error: its mean over independent runs falls
    as N^(-1/2).  eps = 0.1, t = 0.5, both components on a 64 x 64 grid of
    [-3, 3]^2; 16 runs for each N."""
    eps, dt, nsteps = 0.1, 0.005, 100
    mdl = gpu_lq(gpu, paper_system_31(), eps)
    sd = math.sqrt(1.0 - eps)
    g = np.linspace(-3.0, 3.0, 64)
    pts = torch.from_numpy(np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2).copy()).cuda()
    cell = (g[1] - g[0]) ** 2

    def field(n, seed):
        st = gpu.State(n, 2)
        gpu.init_beams(mdl, gpu.make_init_spec(0.0, sd, "normal", 0.0, sd, 0, a0=1.0 / eps), st, seed)
        gpu.step_ensemble(mdl, st, nsteps, dt, seed)
        return gpu.reconstruct(mdl, st, pts).cpu().numpy()[:2] / n

    ref = field(1 << 22, 0x31F00D)
    norm = np.sqrt((np.abs(ref) ** 2).sum() * cell)
    errs = {}
    for n in (100, 400, 1600, 6400):
        e = [np.sqrt((np.abs(field(n, 1000 * n + r) - ref) ** 2).sum() * cell) for r in range(16)]
        errs[n] = float(np.mean(e))
    print("eq:ex1 field: L2 error / L2 norm by N:", {n: round(v / norm, 4) for n, v in errs.items()})
    for n in (100, 400, 1600):
        assert 1.6 <= errs[n] / errs[4 * n] <= 2.5, (n, errs)
    assert errs[6400] < 0.2 * norm
