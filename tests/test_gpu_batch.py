"""Batched persistent launches: many instances in one call.

The batched kernels run the per-beam code of the single-instance kernels, so
a batch must leave every instance bitwise as shgb_step_ensemble would, for
every launch shape; the diag counters must sum over the batch.  A HIP graph
of the batched launch, replayed with eager work in between, must give the
eager results every time.  The autotuner must return one of its candidates.
"""

import numpy as np
import pytest
import torch

from paper_1703_06116_amd import autotune, workloads

from _parity import gpu_model, gpu_spec

pytestmark = pytest.mark.gpu


def instances(d, sizes, seed0=11):
    out = []
    for i, n in enumerate(sizes):
        if d == 1:
            c = workloads.config("qcle1d_1e4", n_beams=n, q_mean=-2.5 - 0.1 * i, q_std=0.3, p_a=28.0 + i,
                                 C=0.004 + 0.001 * i, eps=(0.01, 0.02)[i % 2], seed=seed0 + i)
        else:
            c = workloads.config("qcle12d_2p18", d=d, bath_omega=workloads.bath_omega(d), n_beams=n,
                                 q_mean=-2.5, q_std=0.3, p_a=30.0, C=0.003 + 0.001 * i, seed=seed0 + i)
        out.append(c)
    return out


def fresh_states(gpu, cs, precision):
    states = []
    for i, c in enumerate(cs):
        st = gpu.State(c["n_beams"], 2 * c["d"], precision=precision, beam_id_offset=1000 * i)
        if c["n_beams"]:
            gpu.init_beams(gpu_model(c), gpu_spec(c), st, c["seed"])
        states.append(st)
    return states


def assert_same(a, b):
    for x, y in zip(a, b):
        assert torch.equal(x.f64, y.f64) and torch.equal(x.comp, y.comp) and torch.equal(x.nhop, y.nhop)
        if x.f32 is not None:
            assert torch.equal(x.f32, y.f32)


@pytest.mark.parametrize("d,precision,sizes,nsteps", [
    (1, "fp64", (700, 0, 1, 257, 3000), 300),
    (1, "mixed", (513, 64, 2049), 300),
    (2, "fp64", (37, 5, 130), 200),
    (12, "mixed", (19, 8, 33, 1), 150),
    (12, "fp64", (17, 9), 100),
])
def test_batch_equals_single_instance_calls(gpu, d, precision, sizes, nsteps):
    cs = instances(d, sizes)
    dt = cs[0]["dt"]
    ref = fresh_states(gpu, cs, precision)
    diag_ref = gpu.new_diag()
    for c, st in zip(cs, ref):
        gpu.step_ensemble(gpu_model(c), st, nsteps, dt, c["seed"], diag_ref)
    for cfg in ((4, 2, 1), (2, 1, 4), (4, 4, 4)):
        sts = fresh_states(gpu, cs, precision)
        b = gpu.Batch([gpu_model(c) for c in cs], sts, [c["seed"] for c in cs], config=cfg)
        diag = gpu.new_diag()
        b.step(nsteps, dt, diag)
        assert_same(ref, sts)
        assert torch.equal(diag, diag_ref), (cfg, diag, diag_ref)
    assert diag_ref[0].item() > 0


def test_batch_graph_replays_match_eager(gpu):
    cs = instances(12, (21, 7, 40), seed0=31)
    dt, k = cs[0]["dt"], 40
    models, seeds = [gpu_model(c) for c in cs], [c["seed"] for c in cs]
    eager = fresh_states(gpu, cs, "mixed")
    graphed = fresh_states(gpu, cs, "mixed")
    be = gpu.Batch(models, eager, seeds)
    bg = gpu.Batch(models, graphed, seeds)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):        # warm-up outside the capture, then restore the start state
        bg.step(k, dt)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graphed = fresh_states(gpu, cs, "mixed")
    bg = gpu.Batch(models, graphed, seeds)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bg.step(k, dt)
    for _ in range(3):
        be.step(k, dt)                # eager work between the replays
        g.replay()
        torch.cuda.synchronize()
        assert_same(eager, graphed)
        assert graphed[0].nhop.sum().item() >= 0


def test_autotuner_picks_a_candidate(gpu, tmp_path, monkeypatch):
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    cs = instances(1, (3000, 700))
    states = fresh_states(gpu, cs, "mixed")
    before = [st.f32.clone() for st in states]
    cfg, times = autotune.tune([gpu_model(c) for c in cs], states, [c["seed"] for c in cs], cs[0]["dt"],
                               probe_steps=5, repeats=1)
    assert cfg in autotune.CANDIDATES and len(times) == len(autotune.CANDIDATES)
    assert all(torch.equal(a, st.f32) for a, st in zip(before, states))   # caller's states untouched
    again, _ = autotune.tune([gpu_model(c) for c in cs], states, [c["seed"] for c in cs], cs[0]["dt"])
    assert again == cfg                                                    # from the cache
    assert (tmp_path / "tune.json").exists()
