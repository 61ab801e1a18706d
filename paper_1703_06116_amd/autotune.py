"""Choice of the batched launch shape by measurement.

For a batch (instances of one dimension and precision) the candidates are
every shgb_batch_config of {2, 4} waves per workgroup x {1, 2, 4}
persistent workgroups per compute unit x {1, 4} tiles per queue grab.  Each
is timed with HIP events on a copy of the batch's states over a few
intervals (the copy keeps the caller's states untouched; per-beam results
do not depend on the shape), and the fastest is kept in a JSON cache keyed
by the device, the dimension, the precision and the batch's size class.
"""

import json
import os

import torch

from . import shgb

CANDIDATES = [(w, b, g) for w in (2, 4) for b in (1, 2, 4) for g in (1, 4)]
CACHE_ENV = "SHGB_TUNE_CACHE"


def cache_path():
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.dirname(os.path.abspath(__file__)), ".tune_cache.json")


def _key(states, precision, d):
    beams = sum(st.n for st in states)
    cls = max(beams, 1).bit_length()          # size class: power of two of the total beam count
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return f"{name}|d={d}|{precision}|inst={len(states)}|beams~2^{cls}"


def _clone(st):
    c = shgb.State(st.n, st.m, device=st.f64.device, ld=st.ld, beam_id_offset=st.beam_id_offset,
                   precision=st.precision)
    _copy(c, st)
    return c


def _copy(dst, src):
    dst.f64.copy_(src.f64)
    if src.f32 is not None:
        dst.f32.copy_(src.f32)
    dst.comp.copy_(src.comp)
    dst.nhop.copy_(src.nhop)


def tune(models, states, seeds, dt, probe_steps=20, repeats=2, use_cache=True, log=None):
    """The fastest candidate config for this batch, as a (w, b, g) tuple, and the timings (ms)."""
    d = models[0].d
    precision = states[0].precision
    key = _key(states, precision, d)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
        if key in cache:
            return tuple(cache[key]["config"]), cache[key]["ms"]
    trial = [_clone(st) for st in states]
    times = {}
    for cfg in CANDIDATES:
        b = shgb.Batch(models, trial, seeds, config=cfg)
        for t, st in zip(trial, states):
            _copy(t, st)
        b.step(probe_steps, dt)                       # warm-up (code load, caches)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        best = float("inf")
        for _ in range(repeats):
            for t, st in zip(trial, states):          # every candidate times the same work
                _copy(t, st)
            ev[0].record()
            b.step(probe_steps, dt)
            ev[1].record()
            torch.cuda.synchronize()
            best = min(best, ev[0].elapsed_time(ev[1]))
        times[str(cfg)] = best
        if log:
            log(f"autotune {key} {cfg}: {best:.3f} ms")
    choice = min(CANDIDATES, key=lambda c: times[str(c)])
    cache[key] = {"config": list(choice), "ms": times}
    if use_cache:
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return choice, times
