"""GPU parity of the d-dimensional QCLE path (phase space m = 2d > 2) against the oracle.

One wavefront per beam; d = 2, 3 (small, fast oracle) and d = 12 (the m = 24
workload).  Same bar as the m = 2 path: hop counts and components
bit-exact apart from oracle-reported ties, continuous state within 1e-10
blockwise relative, populations and fields within the rounding scale of
their sums.
"""

import math

import numpy as np
import pytest
import torch

from oracle import observables, shgb as oshgb
from paper_1703_06116_amd import workloads

from _parity import (arrays_from_ensemble, compare_states, ensemble_from_arrays, gpu_model, gpu_spec,
                     oracle_init, oracle_model)

pytestmark = pytest.mark.gpu


def cfg(d, **kw):
    c = workloads.config("qcle12d_2p18", d=d, bath_omega=workloads.bath_omega(d), **kw)
    return c


def crossing(d, n, nsteps):
    return cfg(d, n_beams=n, nsteps=nsteps, q_mean=-2.5, q_std=0.3, p_a=30.0)


@pytest.mark.parametrize("d", [2, 3, 12])
def test_init_matches_oracle(gpu, d):
    c = cfg(d)
    n = 4 * 64 + 13
    st = gpu.State(n, 2 * d, beam_id_offset=77)
    gpu.init_beams(gpu_model(c), gpu_spec(c), st, c["seed"])
    g = gpu.unpack(st)
    e = oracle_init(c, n, 77)
    assert np.abs(g["X"] - e.X).max() <= 1e-13 * np.abs(e.X).max()
    np.testing.assert_array_equal(g["Z"], e.M + 1j * e.N)
    np.testing.assert_array_equal(g["A"], e.A)
    np.testing.assert_allclose(g["E"], e.E, rtol=1e-14)
    # bath modes sampled from their ground-state Wigner widths
    if d == 12:
        w = c["bath_omega"]
        sq = np.sqrt(c["eps"] / (2 * c["mass"] * w))
        assert np.abs(np.std(g["X"][:, 1:d], 0) / sq - 1).max() < 0.35


@pytest.mark.parametrize("d,n,nsteps", [(2, 4 * 37 + 3, 600), (3, 4 * 29 + 1, 600), (12, 4 * 33 + 2, 500)])
def test_step_from_oracle_state(gpu, d, n, nsteps):
    c = crossing(d, n, nsteps)
    e0 = oracle_init(c, n)
    st = gpu.pack(arrays_from_ensemble(e0))
    diag = gpu.new_diag()
    gpu.step_ensemble(gpu_model(c), st, nsteps, c["dt"], c["seed"], diag)
    g = gpu.unpack(st)
    e = e0.subset(np.arange(n))
    oshgb.advance(oracle_model(c), e, nsteps, c["dt"], c["seed"])
    errs, ties = compare_states(g, e, label=f"d={d}")
    d_ = diag.cpu().numpy()
    assert d_[0] == e.nhop.sum() and e.nhop.sum() > n
    assert d_[3] == 0 and d_[4] == 0
    print(f"d={d}", errs, "tie beams", ties)


def test_end_to_end_d12_two_calls(gpu):
    c = crossing(12, 4 * 20 + 3, 400)
    mdl = gpu_model(c)
    st = gpu.State(c["n_beams"], 24)
    gpu.init_beams(mdl, gpu_spec(c), st, c["seed"])
    gpu.step_ensemble(mdl, st, 150, c["dt"], c["seed"])
    gpu.step_ensemble(mdl, st, 250, c["dt"], c["seed"])
    e = oracle_init(c, c["n_beams"])
    oshgb.advance(oracle_model(c), e, 400, c["dt"], c["seed"])
    compare_states(gpu.unpack(st), e, label="d12 e2e")


@pytest.mark.parametrize("d,n", [(2, 1), (2, 4 * 64 + 5), (3, 257), (4, 130), (12, 3 * 64 + 9)])
def test_populations_match_oracle(gpu, d, n):
    c = cfg(d)
    m = 2 * d
    a = workloads.synthetic_ensemble(n, m, seed=n + d, a0=(2 * math.pi * c["eps"]) ** (-m / 2))
    st = gpu.pack(a)
    diag = gpu.new_diag()
    out = gpu.populations(gpu_model(c), st, diag=diag).cpu().numpy()
    e = ensemble_from_arrays(a)
    ref = observables.populations(e, c["eps"])
    ci = observables.beam_integrals(e, c["eps"])
    assert np.abs(out[:, :2] - ref[:, :2]).max() <= 1e-11 * np.abs(ci).sum()
    assert np.abs(out[:, 2:4] - ref[:, 2:4]).max() <= 1e-11 * (np.abs(ci) ** 2).sum()
    np.testing.assert_array_equal(out[:, 4], ref[:, 4])
    assert diag.cpu().numpy()[5] == 0


@pytest.mark.parametrize("d,n,Q", [(2, 70, 300), (3, 9, 257), (12, 4 * 8 + 3, 700)])
def test_reconstruct_matches_oracle(gpu, d, n, Q):
    c = cfg(d)
    m = 2 * d
    a = workloads.synthetic_ensemble(n, m, seed=3 + n, q_range=(0.0, 2.0), p_range=(0.0, 2.0), p_scale=0.3)
    pts = workloads.points_near(a["X"], 0.5 * c["eps"], Q, seed=Q)
    st = gpu.pack(a)
    out = gpu.reconstruct(gpu_model(c), st, torch.from_numpy(pts).cuda()).cpu().numpy()
    e = ensemble_from_arrays(a)
    ref = observables.reconstruct(e, c["eps"], pts)
    scale = observables.reconstruct_abs(e, c["eps"], pts)
    assert (np.abs(out - ref) <= 1e-10 * scale + 1e-300).all()
    assert np.abs(ref).max() > 0


def test_hop_entry_point_d12(gpu):
    c = crossing(12, 4 * 16, 120)
    e0 = oracle_init(c, 64)
    oshgb.advance(oracle_model(c), e0, 120, c["dt"], c["seed"])
    st = gpu.pack(arrays_from_ensemble(e0))
    idx = np.arange(0, 64, 3, dtype=np.int32)
    gpu.hop(gpu_model(c), st, torch.from_numpy(idx).cuda(), c["seed"])
    g = gpu.unpack(st)
    e = e0.subset(np.arange(64))
    oshgb.hop_event(oracle_model(c), e, idx, c["seed"])
    ok = e.dest_ties == 0
    np.testing.assert_array_equal(g["comp"][ok], e.comp[ok])
    np.testing.assert_array_equal(g["phase"][ok], e.phase[ok])
    np.testing.assert_array_equal(g["nhop"], e.nhop)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_empty_and_single_beam_d12(gpu, precision):
    """Edge sizes of the m = 24 path: an empty ensemble gives zero sums everywhere;
    one beam's populations and field (1 and 65 points, ragged against the 64-point
    tiles of the matrix-core kernel) match the oracle on the stored values."""
    c = cfg(12)
    mdl = gpu_model(c)
    st = gpu.State(0, 24, precision=precision)
    gpu.init_beams(mdl, gpu_spec(c), st, c["seed"])
    gpu.step_ensemble(mdl, st, 5, c["dt"], c["seed"])
    assert (gpu.populations(mdl, st).cpu().numpy() == 0).all()
    pts = torch.zeros((7, 24), dtype=torch.float64, device="cuda")
    assert (gpu.reconstruct(mdl, st, pts).cpu().numpy() == 0).all()
    a = workloads.synthetic_ensemble(1, 24, seed=41, q_range=(0.0, 2.0), p_range=(0.0, 2.0), p_scale=0.3)
    st = gpu.pack(a, precision=precision)
    stored = gpu.unpack(st)
    e = ensemble_from_arrays(stored)
    for Q in (1, 65):
        pts = workloads.points_near(a["X"], 0.5 * c["eps"], Q, seed=Q)
        out = gpu.reconstruct(mdl, st, torch.from_numpy(pts).cuda()).cpu().numpy()
        ref = observables.reconstruct(e, c["eps"], pts)
        scale = observables.reconstruct_abs(e, c["eps"], pts)
        assert (np.abs(out - ref) <= 1e-10 * scale + 1e-300).all(), (Q, out, ref)
    pops = gpu.populations(mdl, st).cpu().numpy()
    ref = observables.populations(e, c["eps"])
    ci = observables.beam_integrals(e, c["eps"])
    assert np.abs(pops[:, :2] - ref[:, :2]).max() <= 1e-11 * np.abs(ci).sum()
