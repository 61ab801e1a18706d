"""GPU parity of the one-dimensional QCLE path (phase space m = 2) against the oracle.

Every HIP call goes through the C ABI.  Sizes span several 256-beam blocks
with a ragged tail.  Bar: Philox words, hop counts and components bit-exact
(apart from beams with oracle-reported ties); continuous beam state within
1e-10 blockwise relative; populations and fields within 1e-10 of the scale
of the sum (sum of absolute terms).
"""

import math

import numpy as np
import pytest
import torch

from oracle import observables, philox, shgb as oshgb
from paper_1703_06116_amd import workloads

from _parity import (arrays_from_ensemble, compare_states, ensemble_from_arrays, gpu_model, gpu_spec,
                     oracle_init, oracle_model)

pytestmark = pytest.mark.gpu


def crossing_config(n, nsteps):
    # beams start close to the avoided crossing so that every beam hops within the run
    return workloads.config("qcle1d_1e4", n_beams=n, nsteps=nsteps, q_mean=-2.5, q_std=0.3, p_a=30.0)


def gpu_init(shgb, c, n, offset=0):
    st = shgb.State(n, 2, device="cuda", beam_id_offset=offset)
    shgb.init_beams(gpu_model(c), gpu_spec(c), st, c["seed"])
    return st


def test_philox_words_bit_exact(gpu):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**63, size=(300, 4), dtype=np.int64)
    ctr[:5] = [[0, 0, 0, 0], [1, 2, 3, 4], [-1, -1, -1, -1], [7, 1, philox.TAG_HOP, 0], [9, 0, philox.TAG_NORMAL, 0]]
    seed = 0x1703061160000001
    out = gpu.philox(seed, torch.from_numpy(ctr).cuda()).cpu().numpy()
    for i in range(ctr.shape[0]):
        ref = philox.philox4x64_10([int(x) & (2**64 - 1) for x in ctr[i]], (seed, 0))
        assert [int(x) & (2**64 - 1) for x in out[i]] == list(ref), i


@pytest.mark.parametrize("p_dist", ["normal", "uniform"])
def test_init_matches_oracle(gpu, p_dist):
    c = workloads.config("qcle1d_1e6" if p_dist == "uniform" else "qcle1d_1e4")
    n, off = 1000 + 37, 123456
    g = gpu.unpack(gpu_init(gpu, c, n, off))
    e = oracle_init(c, n, off)
    assert np.abs(g["X"] - e.X).max() <= 1e-13 * np.abs(e.X).max()
    np.testing.assert_array_equal(g["Z"], e.M + 1j * e.N)
    np.testing.assert_array_equal(g["A"], e.A)
    np.testing.assert_array_equal(g["comp"], e.comp)
    assert (g["nhop"] == 0).all() and (g["P"] == 0).all() and (g["S"] == 0).all()
    np.testing.assert_allclose(g["E"], e.E, rtol=1e-14)


def test_step_from_oracle_state(gpu):
    """Stepping alone: the oracle's initial ensemble is the GPU's input."""
    c = crossing_config(2 * 256 + 91, 700)
    e0 = oracle_init(c, c["n_beams"])
    st = gpu.pack(arrays_from_ensemble(e0))
    diag = gpu.new_diag()
    gpu.step_ensemble(gpu_model(c), st, c["nsteps"], c["dt"], c["seed"], diag)
    g = gpu.unpack(st)
    e = e0.subset(np.arange(e0.n))
    oshgb.advance(oracle_model(c), e, c["nsteps"], c["dt"], c["seed"])
    errs, ties = compare_states(g, e, label="step")
    d = diag.cpu().numpy()
    assert d[0] == e.nhop.sum() and e.nhop.sum() > 2 * e.n
    assert d[1] == e.thr_ties.sum() and d[3] == 0 and d[4] == 0
    print("step errors", errs, "tie beams", ties)


def test_end_to_end_init_step(gpu):
    """GPU init + GPU stepping against oracle init + oracle stepping, in two calls."""
    c = crossing_config(3 * 256 + 5, 500)
    st = gpu_init(gpu, c, c["n_beams"])
    gpu.step_ensemble(gpu_model(c), st, 200, c["dt"], c["seed"])
    gpu.step_ensemble(gpu_model(c), st, 300, c["dt"], c["seed"])
    e = oracle_init(c, c["n_beams"])
    oshgb.advance(oracle_model(c), e, 500, c["dt"], c["seed"])
    compare_states(gpu.unpack(st), e, label="e2e")


def test_resume_and_sharding_are_bitwise(gpu):
    c = crossing_config(1000, 300)
    mdl = gpu_model(c)
    whole = gpu_init(gpu, c, 1000)
    gpu.step_ensemble(mdl, whole, 300, c["dt"], c["seed"])
    parts = []
    for off, n in ((0, 613), (613, 387)):
        s = gpu_init(gpu, c, n, off)
        gpu.step_ensemble(mdl, s, 120, c["dt"], c["seed"])
        gpu.step_ensemble(mdl, s, 180, c["dt"], c["seed"])
        parts.append(s)
    a = whole.f64[:, :1000].cpu()
    b = torch.cat([parts[0].f64[:, :613], parts[1].f64[:, :387]], 1).cpu()
    assert torch.equal(a, b)
    assert torch.equal(whole.nhop[:1000].cpu(), torch.cat([parts[0].nhop[:613], parts[1].nhop[:387]]).cpu())


def test_hop_entry_point(gpu):
    c = crossing_config(600, 150)
    e0 = oracle_init(c, 600)
    oshgb.advance(oracle_model(c), e0, 150, c["dt"], c["seed"])   # some beams on every component
    st = gpu.pack(arrays_from_ensemble(e0))
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(600, 257, replace=False)).astype(np.int32)
    idx_dev = torch.from_numpy(np.concatenate([idx, [-1, 600]]).astype(np.int32)).cuda()
    diag = gpu.new_diag()
    gpu.hop(gpu_model(c), st, idx_dev, c["seed"], diag)
    g = gpu.unpack(st)
    e = e0.subset(np.arange(600))
    oshgb.hop_event(oracle_model(c), e, idx, c["seed"])
    ok = e.dest_ties == 0
    np.testing.assert_array_equal(g["comp"][ok], e.comp[ok])
    np.testing.assert_array_equal(g["nhop"], e.nhop)
    np.testing.assert_array_equal(g["phase"][ok], e.phase[ok])
    np.testing.assert_array_equal(g["logw"], e.logw)
    np.testing.assert_array_equal(g["Lam"], e.Lam)
    np.testing.assert_allclose(g["E"], e.E, rtol=1e-14)
    d = diag.cpu().numpy()
    assert d[0] == 257 and d[7] == 2


@pytest.mark.parametrize("n", [1, 255, 3 * 256 + 77])
def test_populations_match_oracle(gpu, n):
    c = workloads.config("qcle1d_1e6")
    a = workloads.synthetic_ensemble(n, 2, seed=n, a0=1.0 / (2 * math.pi * c["eps"]))
    st = gpu.pack(a)
    out = gpu.populations(gpu_model(c), st).cpu().numpy()
    e = ensemble_from_arrays(a)
    ref = observables.populations(e, c["eps"])
    scale = np.abs(observables.beam_integrals(e, c["eps"])).sum()
    assert np.abs(out[:, :2] - ref[:, :2]).max() <= 1e-12 * scale + 1e-300
    sq = np.abs(observables.beam_integrals(e, c["eps"])) ** 2
    assert np.abs(out[:, 2:4] - ref[:, 2:4]).max() <= 1e-12 * sq.sum() + 1e-300
    np.testing.assert_array_equal(out[:, 4], ref[:, 4])
    # bitwise reproducible
    out2 = gpu.populations(gpu_model(c), st).cpu().numpy()
    np.testing.assert_array_equal(out, out2)


@pytest.mark.parametrize("n,Q", [(1, 1), (300, 257), (2 * 256 + 19, 600)])
def test_reconstruct_matches_oracle(gpu, n, Q):
    c = workloads.config("qcle1d_1e6")
    a = workloads.synthetic_ensemble(n, 2, seed=7 + n, q_range=(0.0, 3.0), p_range=(0.0, 3.0),
                                     p_scale=0.5)
    pts = workloads.points_near(a["X"], 4 * c["eps"], Q, seed=Q)
    st = gpu.pack(a)
    out = gpu.reconstruct(gpu_model(c), st, torch.from_numpy(pts).cuda()).cpu().numpy()
    e = ensemble_from_arrays(a)
    ref = observables.reconstruct(e, c["eps"], pts)
    scale = observables.reconstruct_abs(e, c["eps"], pts)
    assert (np.abs(out - ref) <= 1e-10 * scale + 1e-300).all()
    assert np.abs(ref).max() > 0


@pytest.mark.parametrize("extra", [0, 904])
def test_reconstruct_on_a_wide_grid_matches_oracle(gpu, extra):
    # beams spread over the grid as in the bench workload, so that most beam-point terms are
    # exactly zero and whole beams are culled per wavefront; 4096 + 904 points span two sorted
    # point chunks with a ragged tail
    c = workloads.config("qcle1d_1e6")
    n = 3 * 256 + 41
    a = workloads.synthetic_ensemble(n, 2, seed=11, q_range=(10.0, 15.0), p_range=(15.0, 20.0), z_scale=0.3,
                                     p_scale=0.2)
    rng = np.random.default_rng(3)
    pts = np.concatenate([workloads.grid_points_2d(),
                          np.column_stack([rng.uniform(0, 30, extra), rng.uniform(0, 35, extra)])])
    st = gpu.pack(a)
    out = gpu.reconstruct(gpu_model(c), st, torch.from_numpy(pts).cuda()).cpu().numpy()
    e = ensemble_from_arrays(a)
    ref = observables.reconstruct(e, c["eps"], pts)
    scale = observables.reconstruct_abs(e, c["eps"], pts)
    assert (np.abs(out - ref) <= 1e-10 * scale + 1e-300).all()
    assert (ref == 0).mean() > 0.5 and np.abs(ref).max() > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reconstruct_per_point_sums_do_not_depend_on_the_other_points(gpu, precision):
    # each point's sum runs over the beams in one fixed order whatever the other points are:
    # permuting the points, evaluating a subset, or putting non-finite and huge points into
    # the same wavefront (which switches culling off there) leaves every sum bitwise the same
    # (5000 beams give the same beam chunks for every point count used here)
    c = workloads.config("qcle1d_1e6")
    mdl = gpu_model(c)
    st = gpu.State(5000, 2, device="cuda", precision=precision)
    gpu.init_beams(mdl, gpu_spec(c), st, c["seed"])
    gpu.step_ensemble(mdl, st, 400, c["dt"], c["seed"])
    grid = workloads.grid_points_2d()
    ref = gpu.reconstruct(mdl, st, torch.from_numpy(grid).cuda()).cpu().numpy()
    assert np.isfinite(ref).all() and np.abs(ref).max() > 0
    perm = np.random.default_rng(1).permutation(grid.shape[0])
    out = gpu.reconstruct(mdl, st, torch.from_numpy(np.ascontiguousarray(grid[perm])).cuda()).cpu().numpy()
    np.testing.assert_array_equal(out, ref[:, perm])
    sub = np.arange(100, 4096, 7)
    out = gpu.reconstruct(mdl, st, torch.from_numpy(np.ascontiguousarray(grid[sub])).cuda()).cpu().numpy()
    np.testing.assert_array_equal(out, ref[:, sub])
    odd = np.array([[1e120, 3.0], [np.nan, 20.0], [np.inf, 1.0], [-1e300, 1e300]])
    mix = np.concatenate([grid[sub[:30]], odd, grid[sub[30:60]]])
    out = gpu.reconstruct(mdl, st, torch.from_numpy(mix).cuda()).cpu().numpy()
    np.testing.assert_array_equal(out[:, :30], ref[:, sub[:30]])
    np.testing.assert_array_equal(out[:, 34:], ref[:, sub[30:60]])
    assert np.isnan(out[1, 31])   # component 1 (the lower surface) holds beams: NaN propagates
    one = gpu.reconstruct(mdl, st, torch.from_numpy(grid[2080:2081].copy()).cuda()).cpu().numpy()
    np.testing.assert_array_equal(one, ref[:, 2080:2081])


def test_reconstruct_many_sorted_point_chunks(gpu):
    # 20000 scattered points: five Morton-sorted chunks of 4096 and 79 point tiles; each point's
    # sum equals the one from a call on a subset (5000 beams: the same beam chunks for both)
    c = workloads.config("qcle1d_1e6")
    mdl = gpu_model(c)
    st = gpu.State(5000, 2, device="cuda")
    gpu.init_beams(mdl, gpu_spec(c), st, c["seed"])
    gpu.step_ensemble(mdl, st, 400, c["dt"], c["seed"])
    rng = np.random.default_rng(8)
    pts = np.column_stack([rng.uniform(-5, 35, 20000), rng.uniform(0, 40, 20000)])
    out = gpu.reconstruct(mdl, st, torch.from_numpy(pts).cuda()).cpu().numpy()
    sub = np.sort(rng.choice(20000, 3000, replace=False))
    part = gpu.reconstruct(mdl, st, torch.from_numpy(np.ascontiguousarray(pts[sub])).cuda()).cpu().numpy()
    np.testing.assert_array_equal(out[:, sub], part)
    assert np.isfinite(out).all() and (out != 0).any() and (out == 0).any()


def test_empty_and_degenerate(gpu):
    c = workloads.config("qcle1d_1e4")
    mdl = gpu_model(c)
    st = gpu.State(0, 2)
    gpu.init_beams(mdl, gpu_spec(c), st, c["seed"])
    gpu.step_ensemble(mdl, st, 10, c["dt"], c["seed"])
    pops = gpu.populations(mdl, st).cpu().numpy()
    assert (pops == 0).all()
    pts = torch.zeros((5, 2), dtype=torch.float64, device="cuda")
    f = gpu.reconstruct(mdl, st, pts).cpu().numpy()
    assert (f == 0).all()
    # forced hop at once: threshold 0 gives theta = 0 at the interval start
    st = gpu_init(gpu, c, 300)
    e = oracle_init(c, 300)
    st.scal[gpu.State.SCALAR_ROWS["E"], :300] = 0.0
    e.E[:] = 0.0
    st.traj[st.traj_rows()["X"].start, :300] = 0.0       # q = 0: largest coupling
    e.X[:, 0] = 0.0
    gpu.step_ensemble(mdl, st, 3, c["dt"], c["seed"])
    oshgb.advance(oracle_model(c), e, 3, c["dt"], c["seed"])
    compare_states(gpu.unpack(st), e, label="forced")


def test_population_stats_on_the_device(gpu):
    """Sec. 2.4 step 7 on the device: mean and standard error per component from the raw sums
    equal the oracle's from the same sums; several shards' sums added first give the stats of
    the whole ensemble."""
    c = workloads.config("qcle1d_1e6")
    a = workloads.synthetic_ensemble(20001, 2, seed=5, a0=1.0 / (2 * np.pi * c["eps"]))
    st = gpu.pack(a)
    sums = gpu.populations(gpu_model(c), st)
    got = gpu.population_stats(sums, 20001).cpu().numpy()
    mean, se = observables.population_mean_se(sums.cpu().numpy(), 20001)
    ref = np.stack([mean.real, mean.imag, se.real, se.imag], 1)
    assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()
    e = ensemble_from_arrays(a)
    mean_o, se_o = observables.population_mean_se(observables.populations(e, c["eps"]), 20001)
    assert np.abs(got[:, 0] + 1j * got[:, 1] - mean_o).max() <= 1e-12 * np.abs(mean_o).max()
    assert np.abs(got[:, 2] + 1j * got[:, 3] - se_o).max() <= 1e-9 * np.abs(se_o).max()
    one = gpu.population_stats(torch.tensor([[1.0, 2.0, 1.0, 4.0, 1.0]] * 4, dtype=torch.float64, device="cuda"), 1).cpu().numpy()
    assert (one[:, :2] == [1.0, 2.0]).all() and (one[:, 2:] == 0.0).all()
    with pytest.raises(gpu.ShgbError):
        gpu.population_stats(sums, 0)


def test_rk3_scheme_matches_oracle(gpu):
    """Kutta's third-order scheme (the paper's "third-order Runge-Kutta method") on the GPU
    against the oracle run with the same scheme: beams near the crossing, about three hops each,
    per-beam state within 1e-10, hop counts and components bit-exact apart from oracle ties; and
    the scheme changes the result (it is not the RK4 path)."""
    c = workloads.config("qcle1d_1e4", n_beams=300, nsteps=500, q_mean=-2.5, q_std=0.3, p_a=30.0)
    mdl = gpu_model(c)
    st = gpu.State(c["n_beams"], 2)
    gpu.init_beams(mdl, gpu_spec(c), st, c["seed"])
    diag = gpu.new_diag()
    gpu.step_ensemble(mdl, st, c["nsteps"], c["dt"], c["seed"], diag, scheme="rk3")
    e = oracle_init(c, c["n_beams"])
    oshgb.advance(oracle_model(c), e, c["nsteps"], c["dt"], c["seed"], scheme="rk3")
    errs, ties = compare_states(gpu.unpack(st), e, label="rk3")
    assert e.nhop.sum() > 2 * c["n_beams"] and diag[0].item() == e.nhop.sum()
    st4 = gpu.State(c["n_beams"], 2)
    gpu.init_beams(mdl, gpu_spec(c), st4, c["seed"])
    gpu.step_ensemble(mdl, st4, c["nsteps"], c["dt"], c["seed"])
    assert not torch.equal(st4.f64, st.f64)
    with pytest.raises(gpu.ShgbError):
        gpu.step_ensemble(mdl, gpu.State(4, 2, precision="mixed"), 1, 0.5, 1, scheme="rk3")
    print("rk3 errors", errs, "ties", ties)
