"""Benchmark: one pass of the whole SHGB hot path on one MI355X.

A step is: sample the ensemble (init_beams), advance it over every interval
(step_ensemble: RK4 beam ODEs, hop times, hops, weights), reduce the
component populations and sum the field at the evaluation points
(reconstruct), on the 1-D avoided-crossing QCLE workload with 1e6 beams,
4000 intervals of 0.5 and a 64 x 64 (q, p) grid, all in FP64, inputs and
outputs resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config qcle1d_1e6]
                    [--no-cpu-baseline] [--no-mixed]

Prints one JSON line.  `value` is beam-steps per second of the whole FP64
step; the field's beam-point evaluations per second, per-kernel times and
the dominant kernel's roofline figure are reported beside it, with the
stepping kernel's effective HBM rate (`hbm_effective`: the bytes a
step-synchronous kernel would move, one read and one write of the state per
interval, over the fused kernel's time).  The same
workload is then run again on a mixed-precision state (FP32 trajectories,
FP64 phase, rate integral and weights) and reported under "mixed": its
throughput, its speedup over the FP64 path and the largest population
difference between the two runs in units of their combined standard error
(below 1: equal population error).  The CPU baseline times the FP64 oracle
on a bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "beam-steps/s + beam·point evals/s vs FP64 plain path at equal population error"

# FP64 operations per beam-step of the m = 2 stepping kernel, counted from the
# formulas it evaluates (add, multiply, divide, square root and each exp
# count 1; a multiply-add counts 2): 4 right-hand sides of 93 (the adiabatic
# quantities s, s', s'', s''' and d21 of the two-level model from one tanh and
# one Gaussian, 70; the beam right-hand side, 23) plus the Runge-Kutta
# combinations of the 12 integrated doubles (13 each).
FLOPS_PER_BEAM_STEP_M2 = 4 * (70 + 23) + 12 * 13
# per beam-point evaluation of the m = 2 field: y, quadratic form and phase
# (18), exp, sincos (counted 2), complex multiply-accumulate (8)
FLOPS_PER_EVAL_M2 = 18 + 1 + 2 + 8
# FP64 operations per beam-step of the m = 24 wave kernel, counted the same way:
# per right-hand side 3616 (adiabatic quantities 87, Zrr 78 entries x 14 + 3,
# Zrp 144 x 10, Zpp 78 x 4, row/column sums 528, X and P 150, scalars 4) and 13
# per state double for the Runge-Kutta combinations (650 doubles).
FLOPS_PER_BEAM_STEP_M24 = 4 * 3616 + 13 * 650
# per beam-point evaluation of the m = 24 field: the exponent as a contraction over
# F = 325 features for Re and Im (4 F = 1300, the matrix-core work)
FLOPS_PER_EVAL_M24 = 4 * 325
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 64 lanes x 2 flop x 2.4 GHz
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E
# HBM bytes per launch of the FP64 stepping kernel, from rocprofv3 FETCH_SIZE (x2.000) and
# WRITE_SIZE (x1.000), each scaled by what the counter reads for a 1 GiB device copy
# (profiles/step_m2_qcle1d_1e6.md, profiles/step_wave_qcle12d_2p18.md).  Remove an entry when
# its kernel changes.
STEP_TRAFFIC = {
    "qcle1d_1e6": (66680.1 * 2.0 + 133300.8 * 1.0) * 1024,          # step_m2_kernel, 1e6 beams
    "qcle12d_2p18": (2773065.8 * 2.0 + 4688936.7 * 1.0) * 1024,     # step_wave_kernel<12, 32, double>
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="qcle1d_1e6")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run of the same workload (reported beside the FP64 value)")
    ap.add_argument("--cpu-beams", type=int, default=512)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB float64 buffer three times (calibrates the HBM byte counters)")
    return ap.parse_args()


def copy_probe():
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_copy": n * 8, "copies": 3}))


def cpu_baseline(c, n_beams, pts):
    """The FP64 oracle, single process, on n_beams beams of the same workload."""
    import numpy as np
    from oracle import models, observables, sampling, shgb as oshgb
    om = models.QCLE(c["A"], c["B"], c["C"], c["D"], c["mass"], d=c["d"], lam=c["lam"],
                     bath_omega=c["bath_omega"])
    t0 = time.perf_counter()
    ens = sampling.init_beams(om, n_beams, c["eps"], c["seed"], c["q_mean"], c["q_std"], c["p_dist"],
                              c["p_a"], c["p_b"], c["comp0"])
    oshgb.advance(om, ens, c["nsteps"], c["dt"], c["seed"])
    t1 = time.perf_counter()
    observables.populations(ens, c["eps"])
    nq = min(len(pts), 4096)
    t2 = time.perf_counter()
    observables.reconstruct(ens, c["eps"], np.asarray(pts[:nq]))
    t3 = time.perf_counter()
    return {
        "value": n_beams * c["nsteps"] / (t1 - t0),
        "unit": "beam-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n_beams} beams x {c['nsteps']} intervals (init + stepping), then the field of those "
                  f"beams at {nq} points; numpy float64, one process",
        "evals_per_s": n_beams * nq / (t3 - t2),
        "seconds": round(t3 - t0, 2),
    }


def run_batch(a):
    """A batched workload: every instance initialised, advanced by one persistent launch
    (launch shape from the autotuner) and reduced to populations, the whole sequence
    captured once in a HIP graph and replayed; beside it, the same instances through the
    plain FP64 path one instance at a time."""
    import numpy as np
    import torch
    from paper_1703_06116_amd import autotune, shgb, workloads

    cs = workloads.batch_instances(a.config)
    torch.cuda.set_device(0)
    dev = "cuda:0"
    d, nsteps, dt = cs[0]["d"], cs[0]["nsteps"], cs[0]["dt"]
    m = 2 * d
    models = [shgb.make_model(c["d"], c["mass"], c["eps"], c["A"], c["B"], c["C"], c["D"], c["lam"], c["bath_omega"])
              for c in cs]
    specs = [shgb.make_init_spec(c["q_mean"], c["q_std"], c["p_dist"], c["p_a"], c["p_b"], c["comp0"]) for c in cs]
    seeds = [c["seed"] for c in cs]
    N = sum(c["n_beams"] for c in cs)

    def make(precision):
        sts = [shgb.State(c["n_beams"], m, device=dev, precision=precision) for c in cs]
        pops = [torch.empty((4, 5), dtype=torch.float64, device=dev) for _ in cs]
        works = [torch.empty(max(shgb.populations_workspace(c["n_beams"], m), 8), dtype=torch.uint8, device=dev)
                 for c in cs]
        return sts, pops, works

    # mixed precision, batched
    sts, pops, works = make("mixed")
    for mdl, sp, st, sd in zip(models, specs, sts, seeds):
        shgb.init_beams(mdl, sp, st, sd)
    t_tune = time.perf_counter()
    cfg, tune_ms = autotune.tune(models, sts, seeds, dt, probe_steps=10, repeats=1)
    t_tune = time.perf_counter() - t_tune
    batch = shgb.Batch(models, sts, seeds, config=cfg, device=dev)

    def batched_step():
        for mdl, sp, st, sd in zip(models, specs, sts, seeds):
            shgb.init_beams(mdl, sp, st, sd)
        batch.step(nsteps, dt)
        for mdl, st, p, w in zip(models, sts, pops, works):
            shgb.populations(mdl, st, out=p, work=w)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(max(a.warmup, 1)):
            batched_step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched_step()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for _ in range(a.steps):
        graph.replay()
    ev[1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    graph_ms = ev[0].elapsed_time(ev[1]) / a.steps
    mix = [shgb.population_mean_se(p.cpu().numpy(), c["n_beams"]) for p, c in zip(pops, cs)]
    del graph, batch, sts, pops, works
    torch.cuda.empty_cache()

    # plain FP64 path, one instance at a time
    sts64, pops64, works64 = make("fp64")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for mdl, sp, st, sd, p, w, c in zip(models, specs, sts64, seeds, pops64, works64, cs):
        shgb.init_beams(mdl, sp, st, sd)
        shgb.step_ensemble(mdl, st, nsteps, dt, sd)
        shgb.populations(mdl, st, out=p, work=w)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    f64 = [shgb.population_mean_se(p.cpu().numpy(), c["n_beams"]) for p, c in zip(pops64, cs)]
    worst = 0.0
    for (mm, sm), (m6, s6) in zip(mix, f64):
        se = np.sqrt(np.abs(sm) ** 2 + np.abs(s6) ** 2)
        worst = max(worst, float((np.abs(mm - m6) / np.maximum(se, 1e-300)).max()))
    value = N * nsteps / (ms_per_step / 1e3)
    line = {
        "metric": METRIC, "value": value, "unit": "beam-steps/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 trajectories + f64 phase/weights", "data": "synthetic",
        "config": {"workload": a.config, "system": f"qcle-two-level-{d}d", "instances": len(cs), "n_beams": N,
                   "intervals": nsteps, "dt": dt, "phase_space_dim": m, "parallelism": "none (1 GPU)"},
        "graph_ms_per_step": graph_ms,
        "launch_shape": {"waves_per_block": cfg[0], "blocks_per_cu": cfg[1], "tiles_per_grab": cfg[2]},
        "autotune_s": t_tune, "autotune_ms": tune_ms,
        "fp64_per_instance": {"value": N * nsteps / (t3 - t2), "ms_per_step": (t3 - t2) * 1e3,
                              "unit": "beam-steps/s"},
        "speedup_vs_fp64_per_instance": (t3 - t2) * 1e3 / ms_per_step,
        "population_diff_over_se": worst,
    }
    print(json.dumps(line), flush=True)


def run_grad(a, c):
    """The derivative workload: the ensemble sampled, then its populations and their derivatives
    along all five theta directions (five tangent passes over every interval); beside it the plain
    FP64 forward run of the same ensemble (init, step, populations)."""
    import numpy as np
    import torch
    from paper_1703_06116_amd import shgb

    N, nsteps, dt, seed, m = c["n_beams"], c["nsteps"], c["dt"], c["seed"], 2 * c["d"]
    mdl = shgb.make_model(c["d"], c["mass"], c["eps"], c["A"], c["B"], c["C"], c["D"], c["lam"], c["bath_omega"])
    spec = shgb.make_init_spec(c["q_mean"], c["q_std"], c["p_dist"], c["p_a"], c["p_b"], c["comp0"])
    dev = "cuda:0"
    torch.cuda.set_device(0)
    st = shgb.State(N, m, device=dev)
    out = torch.zeros((5, 4, 4), dtype=torch.float64, device=dev)
    work = torch.empty(max(shgb.population_tangent_workspace(N), 8), dtype=torch.uint8, device=dev)
    diag = shgb.new_diag(dev)
    pops = torch.empty((4, 5), dtype=torch.float64, device=dev)
    pop_work = torch.empty(max(shgb.populations_workspace(N, m), 8), dtype=torch.uint8, device=dev)

    def grad_step():
        shgb.init_beams(mdl, spec, st, seed)
        shgb.population_tangent(mdl, st, nsteps, dt, seed, out=out, work=work, diag=diag)

    def forward_step():
        shgb.init_beams(mdl, spec, st, seed)
        shgb.step_ensemble(mdl, st, nsteps, dt, seed)
        shgb.populations(mdl, st, out=pops, work=pop_work)

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / a.steps

    ms_grad = timed(grad_step)
    o = out.cpu().numpy()
    ms_fwd = timed(forward_step)
    p = pops.cpu().numpy()
    value_diff = float(np.abs(o[0, :, 0] - p[:, 0]).max() / max(np.abs(p[:, 0]).sum(), 1e-300))
    line = {
        "metric": METRIC, "value": N * nsteps / (ms_grad / 1e3), "unit": "beam-steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_grad, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (value, derivative) pairs", "data": "synthetic",
        "config": {"workload": a.config, "system": f"qcle-two-level-{c['d']}d", "n_beams": N, "intervals": nsteps,
                   "dt": dt, "eps": c["eps"], "phase_space_dim": m, "directions": 5,
                   "parallelism": "none (1 GPU)"},
        "note": "value counts each beam-step once for all five directions (five tangent passes)",
        "forward_fp64_ms_per_step": ms_fwd,
        "gradient_over_forward": ms_grad / ms_fwd,
        "upper_population": float(o[0, 0, 0] / N),
        "d_upper_population": {n: float(o[j, 0, 2] / N) for j, n in enumerate(("A", "B", "C", "D", "p_mean"))},
        "tangent_values_vs_forward_rel": value_diff,
        "diag": {n: int(v) for n, v in zip(shgb.DIAG_NAMES, diag.cpu().numpy() // max(a.steps + a.warmup, 1))},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {a.gpus}). "
              "Beams are independent; a multi-GPU run would shard beams and sum the tallies once.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1703_06116_amd import shgb, workloads

    if a.config in workloads.BATCH:
        return run_batch(a)
    c = workloads.config(a.config)
    if a.config in workloads.GRADIENT:
        return run_grad(a, c)
    N, nsteps, dt, seed, m = c["n_beams"], c["nsteps"], c["dt"], c["seed"], 2 * c["d"]
    if m not in (2, 24):
        raise SystemExit("bench.py drives the m = 2 and m = 24 workloads")
    mdl = shgb.make_model(c["d"], c["mass"], c["eps"], c["A"], c["B"], c["C"], c["D"], c["lam"],
                          c["bath_omega"])
    spec = shgb.make_init_spec(c["q_mean"], c["q_std"], c["p_dist"], c["p_a"], c["p_b"], c["comp0"])
    dev = "cuda:0"
    torch.cuda.set_device(0)
    pts_np = workloads.grid_points_2d() if m == 2 else workloads.points_near_final(c, c["n_points"], seed=3)
    Q = pts_np.shape[0] if c["n_points"] else 0
    pts = torch.from_numpy(pts_np[:Q]).to(dev)
    names = ("init", "step", "populations", "reconstruct")

    def timed_run(precision, steps, warmup):
        """warmup + steps bench steps on one state of the given precision."""
        st = shgb.State(N, m, device=dev, precision=precision)
        diag = shgb.new_diag(dev)
        pops = torch.empty((4, 5), dtype=torch.float64, device=dev)
        pop_work = torch.empty(max(shgb.populations_workspace(N, m), 8), dtype=torch.uint8, device=dev)
        rec = torch.empty((4, Q, 2), dtype=torch.float64, device=dev)
        rec_work = torch.empty(max(shgb.reconstruct_workspace(N, m, Q), 8), dtype=torch.uint8, device=dev)

        def one_step(evs=None):
            def mark(i):
                if evs is not None:
                    evs[i].record()
            mark(0)
            shgb.init_beams(mdl, spec, st, seed)
            mark(1)
            shgb.step_ensemble(mdl, st, nsteps, dt, seed, diag)
            mark(2)
            shgb.populations(mdl, st, out=pops, work=pop_work)
            mark(3)
            if Q:
                shgb.reconstruct(mdl, st, pts, out=rec, work=rec_work)
            mark(4)

        for _ in range(warmup):
            one_step()
        torch.cuda.synchronize()
        diag.zero_()
        events = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            one_step(events[k])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        phase_ms = {n: float(np.mean([events[k][i].elapsed_time(events[k][i + 1]) for k in range(steps)]))
                    for i, n in enumerate(names)}
        mean, se = shgb.population_mean_se(pops.cpu().numpy(), N)
        field = rec.cpu().numpy() if Q else None
        del st, rec_work, pop_work
        return dict(ms_per_step=(t1 - t0) * 1e3 / steps, phase_ms=phase_ms, mean=mean, se=se,
                    diag=diag.cpu().numpy() // max(steps, 1), field=field)

    r64 = timed_run("fp64", a.steps, a.warmup)
    ms_per_step, phase_ms = r64["ms_per_step"], r64["phase_ms"]
    value = N * nsteps / (ms_per_step / 1e3)
    evals_per_s = N * Q / (phase_ms["reconstruct"] / 1e3) if Q else None
    fps = FLOPS_PER_BEAM_STEP_M2 if m == 2 else FLOPS_PER_BEAM_STEP_M24
    fpe = FLOPS_PER_EVAL_M2 if m == 2 else FLOPS_PER_EVAL_M24
    step_tflops = fps * N * nsteps / (phase_ms["step"] / 1e3) / 1e12
    mean, se, d = r64["mean"], r64["se"], r64["diag"]
    mixed = None
    if not a.no_mixed:
        rmx = timed_run("mixed", a.steps, a.warmup)
        se_pair = np.sqrt(np.abs(se) ** 2 + np.abs(rmx["se"]) ** 2)
        dmx = rmx["diag"]
        mixed = {
            "precision": "trajectories and Hessians FP32; S, Lam, thresholds, weights, populations FP64; "
                         + ("field FP32 with FP64 sums" if m == 2 else "field FP64 from FP32-stored beams"),
            "value": N * nsteps / (rmx["ms_per_step"] / 1e3), "unit": "beam-steps/s",
            "ms_per_step": rmx["ms_per_step"], "kernel_ms": rmx["phase_ms"],
            "beam_point_evals_per_s": N * Q / (rmx["phase_ms"]["reconstruct"] / 1e3) if Q else None,
            "speedup_vs_fp64": ms_per_step / rmx["ms_per_step"],
            "step_speedup_vs_fp64": phase_ms["step"] / rmx["phase_ms"]["step"],
            "population_diff_over_se": float((np.abs(rmx["mean"] - mean) / np.maximum(se_pair, 1e-300)).max()),
            "field_rel_l2_vs_fp64": (None if not Q else
                                     float(np.linalg.norm(rmx["field"] - r64["field"]) /
                                           max(np.linalg.norm(r64["field"]), 1e-300))),
            "diag_per_step": {n: int(v) for n, v in zip(shgb.DIAG_NAMES, dmx)},
        }

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "beam-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.config, "system": f"qcle-two-level-{c['d']}d", "n_beams": N, "intervals": nsteps,
                   "dt": dt, "eps": c["eps"], "eval_points": Q, "phase_space_dim": m,
                   "parallelism": "none (1 GPU)"},
        "beam_point_evals_per_s": evals_per_s,
        "kernel_ms": phase_ms,
        "roofline": {"bound": "alu", "kernel": "step_m2_kernel" if m == 2 else "step_wave_kernel<12>",
                     "achieved": step_tflops,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": step_tflops / PEAK_FP64_TFLOPS,
                     "traffic": STEP_TRAFFIC.get(a.config), "traffic_unit": "bytes/launch",
                     # the state a call reads and writes once: X, P, Z, S, Lam, logw, phase, E
                     # (A is constant for the QCLE, gamma_ll = 0) and comp, nhop
                     "algorithmic_bytes": 2 * (8 * (2 * m + m * (m + 1) + 6) + 8) * N,
                     "flops_per_unit": fps, "units_per_launch": N * nsteps},
        # the stepping kernel keeps the state on chip for all intervals; against a step-synchronous
        # kernel that reads and writes the state once per interval its rate is an effective bandwidth
        "hbm_effective": {"bytes_per_beam_step_unfused": 2 * (8 * (2 * m + m * (m + 1) + 6) + 8),
                          "achieved": 2 * (8 * (2 * m + m * (m + 1) + 6) + 8) * N * nsteps
                          / (phase_ms["step"] / 1e3) / 1e9,
                          "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                          "frac": 2 * (8 * (2 * m + m * (m + 1) + 6) + 8) * N * nsteps
                          / (phase_ms["step"] / 1e3) / 1e9 / PEAK_HBM_GBPS},
        "reconstruct_roofline": ({"bound": "alu" if m == 2 else "mfma", "achieved": fpe * evals_per_s / 1e12,
                                  "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                  "frac": fpe * evals_per_s / 1e12 / PEAK_FP64_TFLOPS,
                                  "flops_per_unit": fpe,
                                  # m = 2: the kernel culls the beam-point pairs whose term is exactly zero
                                  # (same sums); the rate counts every pair of the direct sum
                                  "note": ("per beam-point pair of the direct sum, exactly-zero terms culled"
                                           if m == 2 else "per beam-point pair")}
                                 if Q else None),
        "populations": {"mean_re": mean.real.tolist(), "mean_im": mean.imag.tolist(),
                        "se_re": se.real.tolist()},
        "diag_per_step": {n: int(v) for n, v in zip(shgb.DIAG_NAMES, d)},
        "mixed": mixed,
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c, a.cpu_beams, pts_np)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
