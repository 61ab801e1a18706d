"""Benchmark: one pass of the whole SHGB hot path on one MI355X.

A step is: sample the ensemble (init_beams), advance it over every interval
(step_ensemble: RK4 beam ODEs, hop times, hops, weights), reduce the
component populations and sum the field at the evaluation points
(reconstruct), on the 1-D avoided-crossing QCLE workload with 1e6 beams,
4000 intervals of 0.5 and a 64 x 64 (q, p) grid, all in FP64, inputs and
outputs resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
                    [--no-cpu-baseline] [--no-mixed] [--no-extra]

Prints one JSON line.  `value` is beam-steps per second of the whole FP64
step; the field's beam-point evaluations per second, per-kernel times (HIP
events on the launch stream) and the dominant kernel's roofline figure are
reported beside it.  The same workload is run again on a mixed-precision
state ("mixed": FP32 trajectories, FP64 phase, rate integral and weights;
its speedup and the population difference in standard errors, below 1 =
equal population error).  Beside the headline, with a bounded number of
steps each, the other workloads of the hot path (omit with --no-extra):
"c3" the d = 12 (m = 24) ensemble with its matrix-core field, FP64 and
mixed; "c4" the 64-instance batch in one persistent launch replayed from a
HIP graph, against the FP64 per-instance path; "c5" the gradient of the
upper population in five parameters (checkpointed forward + one reverse
sweep) against the plain forward run.  Each block carries the roofline of
its dominant kernel and a CPU baseline: the FP64 oracle on a bounded sample
of the same workload, sharded over the host cores (one process and one BLAS
thread per core), run before the GPU work.

--config NAME runs one workload alone (its block as the whole line).
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "beam-steps/s + beam·point evals/s vs FP64 plain path at equal population error"
HEADLINE = "qcle1d_1e6"

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
# FP64 operations per beam-interval of the m = 24 reverse kernel: four vector-Jacobian
# products of the right-hand side (each as costly as the right-hand side without its
# two-level quantities, 3616 - 87, plus 62 for the cotangents of those quantities and their
# pullback through the 5 x 5 Jacobian), the Jacobian itself once per step (five directional
# derivatives, 2 x 87 each) and the reverse Runge-Kutta combinations (4 per state double and
# stage); a reverse sweep that runs each segment again adds the replay's RK4 step (22914)
FLOPS_PER_BEAM_STEP_REV_M24 = 4 * (3616 - 87 + 62) + 5 * 2 * 87 + 16 * 650
FLOPS_PER_BEAM_STEP_ADJ_M24 = FLOPS_PER_BEAM_STEP_M24 + FLOPS_PER_BEAM_STEP_REV_M24
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector and FP64 matrix: 256 CU x 64 lanes x 2 flop x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E
# HBM bytes per launch of the FP64 stepping kernels, from rocprofv3 FETCH_SIZE (x2.000) and
# WRITE_SIZE (x1.000), each scaled by what the counter reads for a 1 GiB device copy
# (profiles/step_m2_qcle1d_1e6.md, profiles/step_wave_qcle12d_2p18.md).  Each entry names the
# kernel it was taken on; remove it when that kernel changes.
STEP_TRAFFIC = {
    "qcle1d_1e6": ((66703.4 * 2.0 + 133300.8 * 1.0) * 1024,
                   "step_m2_kernel (per-lane interval calls, three waves per SIMD), "
                   "profiles/step_m2_qcle1d_1e6.md"),
    "qcle12d_2p18": ((672048.0 * 2.0 + 1658031.0 * 1.0) * 1024,
                     "step_wave_kernel<12, 32, double> (two wavefronts per SIMD, no scratch, the tile's rows "
                     "written through LDS), profiles/step_wave_qcle12d_2p18.md"),
}
# Fraction of the direct sum's VALU instructions that the culled m = 2 field kernel executes
# on the bench grid (SQ_INSTS_VALU 1.29e9 culled against 4.01e9 direct,
# profiles/step_m2_qcle1d_1e6.md): the executed-work utilisation is the direct-sum rate over this.
RECON_M2_EXECUTED_FRACTION = 1.29 / 4.01


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run of the same workload (reported beside the FP64 value)")
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload")
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


# ---------------------------------------------------------------------------
# CPU baselines: the oracle on bounded samples, sharded over the host cores
# (fork workers started before the GPU is touched; one BLAS thread each).

def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def host_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_model(c):
    from oracle import models
    return models.QCLE(c["A"], c["B"], c["C"], c["D"], c["mass"], d=c["d"], lam=c.get("lam", 0.0),
                       bath_omega=c["bath_omega"])


def _shard_run(args):
    """One worker: sample beams [off, off + n) of config c and step them; returns seconds."""
    c, n, off, nsteps = args
    from threadpoolctl import threadpool_limits
    from oracle import sampling, shgb as oshgb
    with threadpool_limits(1):
        om = _oracle_model(c)
        t0 = time.perf_counter()
        ens = sampling.init_beams(om, n, c["eps"], c["seed"], c["q_mean"], c["q_std"], c["p_dist"], c["p_a"],
                                  c["p_b"], c["comp0"], beam_id_offset=off)
        oshgb.advance(om, ens, nsteps, c["dt"], c["seed"])
        return time.perf_counter() - t0


def _field_run(args):
    c, n, pts = args
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import observables, sampling
    with threadpool_limits(1):
        om = _oracle_model(c)
        ens = sampling.init_beams(om, n, c["eps"], c["seed"], c["q_mean"], c["q_std"], c["p_dist"], c["p_a"],
                                  c["p_b"], c["comp0"])
        t0 = time.perf_counter()
        observables.reconstruct(ens, c["eps"], np.asarray(pts))
        return time.perf_counter() - t0


def _cd_run(args):
    """One oracle run of the derivative sample at theta shifted along direction j by s h."""
    c, n, j, s = args
    from threadpoolctl import threadpool_limits
    from oracle import observables, sampling, shgb as oshgb
    with threadpool_limits(1):
        c = dict(c)
        th = [c["A"], c["B"], c["C"], c["D"], c["p_a"]]
        if j >= 0:
            th[j] += s * 1e-6 * abs(th[j])
        c.update(A=th[0], B=th[1], C=th[2], D=th[3], p_a=th[4])
        om = _oracle_model(c)
        t0 = time.perf_counter()
        ens = sampling.init_beams(om, n, c["eps"], c["seed"], c["q_mean"], c["q_std"], c["p_dist"], c["p_a"],
                                  c["p_b"], c["comp0"])
        oshgb.advance(om, ens, c["nsteps"], c["dt"], c["seed"])
        p = observables.populations(ens, c["eps"])
        return time.perf_counter() - t0, float(p[0, 0])


def cpu_baselines(names, pool):
    """CPU baselines of the named workloads (the oracle timed on the host cores)."""
    from paper_1703_06116_amd import workloads
    cores, model = host_cores(), host_model()
    out = {}

    def sharded(c, per_core, nsteps, what):
        jobs = [(c, per_core, k * per_core, nsteps) for k in range(cores)]
        t0 = time.perf_counter()
        pool.map(_shard_run, jobs)
        wall = time.perf_counter() - t0
        n = per_core * cores
        return {"value": n * nsteps / wall, "unit": "beam-steps/s", "cores": cores, "cpu_model": model,
                "kind": "oracle", "seconds": round(wall, 2),
                "sample": f"{n} beams x {nsteps} intervals ({per_core} per core, {cores} worker processes, "
                          f"one BLAS thread each){what}; numpy float64"}

    for name in names:
        if name == "qcle1d_1e6":
            c = workloads.config(name)
            r = sharded(c, 768, c["nsteps"], "")
            pts = workloads.grid_points_2d()
            t0 = time.perf_counter()
            pool.map(_field_run, [(c, 64, pts)] * cores)
            wall = time.perf_counter() - t0
            r["evals_per_s"] = 64 * cores * len(pts) / wall
            r["sample"] += f"; field: {64 * cores} beams x {len(pts)} grid points, {cores} processes"
            out[name] = r
        elif name == "qcle12d_2p18":
            c = workloads.config(name)
            out[name] = sharded(c, 128, c["nsteps"], "")
        elif name == "batch64_d12":
            cs = workloads.batch_instances(name)
            jobs = [(cs[i], 256, 0, cs[i]["nsteps"]) for i in range(0, len(cs), max(1, len(cs) // cores))][:cores]
            t0 = time.perf_counter()
            pool.map(_shard_run, jobs)
            wall = time.perf_counter() - t0
            n = 256 * len(jobs)
            out[name] = {"value": n * cs[0]["nsteps"] / wall, "unit": "beam-steps/s", "cores": len(jobs),
                         "cpu_model": model, "kind": "oracle", "seconds": round(wall, 2),
                         "sample": f"256 beams of each of {len(jobs)} instances x {cs[0]['nsteps']} intervals, "
                                   "FP64, one process per instance"}
        elif name == "qcle12d_grad":
            c = workloads.config(name)
            n = 96
            jobs = [(c, n, -1, 0)] + [(c, n, j, s) for j in range(5) for s in (1, -1)]
            t0 = time.perf_counter()
            pool.map(_cd_run, jobs)
            wall = time.perf_counter() - t0
            out[name] = {"value": n * c["nsteps"] / wall, "unit": "beam-steps/s (of the five-parameter gradient)",
                         "cores": min(cores, len(jobs)), "cpu_model": model, "kind": "oracle",
                         "seconds": round(wall, 2),
                         "sample": f"central differences of the oracle (h = 1e-6 relative, common random numbers): "
                                   f"{len(jobs)} runs of {n} beams x {c['nsteps']} intervals, one process each"}
    return out


# ---------------------------------------------------------------------------
# GPU workloads

def _timer():
    import torch
    return torch.cuda.Event(enable_timing=True)


def run_plain(name, steps, warmup, with_mixed):
    """init + step + populations + field on one state, FP64 (and mixed)."""
    import numpy as np
    import torch
    from paper_1703_06116_amd import shgb, workloads

    c = workloads.config(name)
    N, nsteps, dt, seed, m = c["n_beams"], c["nsteps"], c["dt"], c["seed"], 2 * c["d"]
    mdl = shgb.make_model(c["d"], c["mass"], c["eps"], c["A"], c["B"], c["C"], c["D"], c["lam"], c["bath_omega"])
    spec = shgb.make_init_spec(c["q_mean"], c["q_std"], c["p_dist"], c["p_a"], c["p_b"], c["comp0"])
    dev = "cuda:0"
    pts_np = workloads.grid_points_2d() if m == 2 else workloads.points_near_final(c, c["n_points"], seed=3)
    Q = pts_np.shape[0] if c["n_points"] else 0
    pts = torch.from_numpy(pts_np[:Q]).to(dev)
    names = ("init", "step", "populations", "reconstruct")

    def timed_run(precision):
        st = shgb.State(N, m, device=dev, precision=precision)
        diag = shgb.new_diag(dev)
        pops = torch.empty((4, 5), dtype=torch.float64, device=dev)
        stats = torch.empty((4, 4), dtype=torch.float64, device=dev)
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
            shgb.population_stats(pops, N, out=stats)
            mark(3)
            if Q:
                shgb.reconstruct(mdl, st, pts, out=rec, work=rec_work)
            mark(4)

        for _ in range(warmup):
            one_step()
        torch.cuda.synchronize()
        diag.zero_()
        events = [[_timer() for _ in range(5)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            one_step(events[k])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        phase_ms = {n: float(np.mean([events[k][i].elapsed_time(events[k][i + 1]) for k in range(steps)]))
                    for i, n in enumerate(names)}
        s = stats.cpu().numpy()
        field = rec.cpu().numpy() if Q else None
        f32 = None
        if precision == "mixed" and m == 24 and Q:
            # the same field on the FP32 matrix cores (error stated, not the default)
            w32 = torch.empty(max(shgb.reconstruct_workspace(N, m, Q, "fp32"), 8), dtype=torch.uint8, device=dev)
            r32 = torch.empty((4, Q, 2), dtype=torch.float64, device=dev)
            shgb.reconstruct(mdl, st, pts, out=r32, work=w32, mode="fp32")
            ev = [_timer() for _ in range(2)]
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(steps):
                shgb.reconstruct(mdl, st, pts, out=r32, work=w32, mode="fp32")
            ev[1].record()
            torch.cuda.synchronize()
            f32_ms = ev[0].elapsed_time(ev[1]) / steps
            v32 = r32.cpu().numpy()
            f32 = {"ms": f32_ms, "evals_per_s": N * Q / (f32_ms / 1e3),
                   "speedup_vs_fp64_matrix_field": phase_ms["reconstruct"] / f32_ms,
                   "rel_l2_vs_fp64_matrix_field": float(np.linalg.norm(v32 - field) / max(np.linalg.norm(field),
                                                                                           1e-300)),
                   "roofline": {"bound": "mfma", "kernel": "rm32_gemm_kernel (FP32 MFMA 16x16x4)",
                                "achieved": FLOPS_PER_EVAL_M24 * N * Q / (f32_ms / 1e3) / 1e12,
                                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                "frac": FLOPS_PER_EVAL_M24 * N * Q / (f32_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
                                "note": "whole field call (beam weights, GEMM, reduction) against the FP32 matrix "
                                        "peak"},
                   "stated_error": "1e-3 of sum |terms| at worst, 1e-4 relative L2 against the FP64 oracle "
                                   "(tests/test_gpu_field32.py)"}
            del w32, r32
        del st, rec_work, pop_work
        torch.cuda.empty_cache()
        return dict(ms_per_step=(t1 - t0) * 1e3 / steps, phase_ms=phase_ms, mean=s[:, 0] + 1j * s[:, 1],
                    se=s[:, 2] + 1j * s[:, 3], diag=diag.cpu().numpy() // max(steps, 1), field=field, f32=f32)

    r64 = timed_run("fp64")
    ms_per_step, phase_ms = r64["ms_per_step"], r64["phase_ms"]
    evals_per_s = N * Q / (phase_ms["reconstruct"] / 1e3) if Q else None
    fps = FLOPS_PER_BEAM_STEP_M2 if m == 2 else FLOPS_PER_BEAM_STEP_M24
    fpe = FLOPS_PER_EVAL_M2 if m == 2 else FLOPS_PER_EVAL_M24
    step_tflops = fps * N * nsteps / (phase_ms["step"] / 1e3) / 1e12
    mean, se, d = r64["mean"], r64["se"], r64["diag"]
    traffic = STEP_TRAFFIC.get(name)
    unfused = 2 * (8 * (2 * m + m * (m + 1) + 6) + 8)
    line = {
        "value": N * nsteps / (ms_per_step / 1e3), "unit": "beam-steps/s", "ms_per_step": ms_per_step,
        "steps": steps, "warmup": warmup, "dtype": "f64",
        "config": {"workload": name, "system": f"qcle-two-level-{c['d']}d", "n_beams": N, "intervals": nsteps,
                   "dt": dt, "eps": c["eps"], "eval_points": Q, "phase_space_dim": m},
        "beam_point_evals_per_s": evals_per_s,
        "kernel_ms": phase_ms,
        "roofline": {"bound": "alu", "kernel": "step_m2_kernel" if m == 2 else "step_wave_kernel<12, 32, double>",
                     "achieved": step_tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": step_tflops / PEAK_FP64_TFLOPS,
                     "traffic": traffic[0] if traffic else None, "traffic_unit": "bytes/launch",
                     "traffic_source": ("rocprofv3 FETCH_SIZE/WRITE_SIZE scaled by a 1 GiB copy, " + traffic[1])
                     if traffic else None,
                     # the state one call reads and writes once: X, P, Z, S, Lam, logw, phase, E (A is constant
                     # for the QCLE, gamma_ll = 0) and comp, nhop
                     "algorithmic_bytes": unfused * N, "flops_per_unit": fps, "units_per_launch": N * nsteps,
                     "peak_note": "FP64 vector issue: 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz"},
        # the stepping kernel keeps each beam's state on chip for all intervals: against a
        # step-synchronous kernel (one read and one write of the state per interval) its rate is an
        # effective bandwidth, above the HBM peak; not a roofline fraction
        "hbm_effective_not_roofline": {"bytes_per_beam_step_unfused": unfused,
                                       "effective_GBps": unfused * N * nsteps / (phase_ms["step"] / 1e3) / 1e9,
                                       "hbm_peak_GBps": PEAK_HBM_GBPS},
        "populations": {"mean_re": mean.real.tolist(), "mean_im": mean.imag.tolist(), "se_re": se.real.tolist()},
        "diag_per_step": {n: int(v) for n, v in zip(shgb.DIAG_NAMES, d)},
    }
    if Q:
        direct = fpe * evals_per_s / 1e12
        if m == 2:
            line["reconstruct_roofline"] = {
                "bound": "alu", "kernel": "recon_m2_kernel", "unit": "TFLOP/s", "peak": PEAK_FP64_TFLOPS,
                "flops_per_unit": fpe,
                "executed": direct * RECON_M2_EXECUTED_FRACTION,
                "executed_frac": direct * RECON_M2_EXECUTED_FRACTION / PEAK_FP64_TFLOPS,
                "direct_sum_equivalent": direct, "direct_sum_equivalent_frac": direct / PEAK_FP64_TFLOPS,
                "note": "the kernel culls beam-point pairs whose term is exactly zero (same sums): executed work "
                        "is the direct sum's times the culled/direct VALU instruction ratio "
                        f"{RECON_M2_EXECUTED_FRACTION:.3f} (profiles/step_m2_qcle1d_1e6.md)"}
        else:
            line["reconstruct_roofline"] = {
                "bound": "mfma", "kernel": "rm_gemm_kernel (FP64 MFMA 4x4x4)", "achieved": direct,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": direct / PEAK_FP64_TFLOPS,
                "flops_per_unit": fpe, "units_per_launch": N * Q,
                "note": "time of the whole field call (feature kernels, GEMM, reduction): a lower bound on the "
                        "GEMM kernel's rate"}
    if with_mixed:
        rmx = timed_run("mixed")
        se_pair = np.sqrt(np.abs(se) ** 2 + np.abs(rmx["se"]) ** 2)
        line["mixed"] = {
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
            "diag_per_step": {n: int(v) for n, v in zip(shgb.DIAG_NAMES, rmx["diag"])},
        }
        if rmx["f32"] is not None:
            line["mixed"]["field_fp32_matrix"] = rmx["f32"]
    return line


def run_batch(name, steps, warmup):
    """A batched workload: every instance initialised, advanced by one persistent launch
    (launch shape from the autotuner) and reduced to populations, the whole sequence
    captured once in a HIP graph and replayed; beside it, the same instances through the
    plain FP64 path one instance at a time."""
    import numpy as np
    import torch
    from paper_1703_06116_amd import autotune, shgb, workloads

    cs = workloads.batch_instances(name)
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
        for _ in range(max(warmup, 1)):
            batched_step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched_step()
    ev = [_timer() for _ in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for _ in range(steps):
        graph.replay()
    ev[1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    graph_ms = ev[0].elapsed_time(ev[1]) / steps
    mix = [shgb.population_mean_se(p, c["n_beams"]) for p, c in zip(pops, cs)]
    del graph, batch, sts, pops, works
    torch.cuda.empty_cache()

    sts64, pops64, works64 = make("fp64")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for mdl, sp, st, sd, p, w in zip(models, specs, sts64, seeds, pops64, works64):
        shgb.init_beams(mdl, sp, st, sd)
        shgb.step_ensemble(mdl, st, nsteps, dt, sd)
        shgb.populations(mdl, st, out=p, work=w)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    f64 = [shgb.population_mean_se(p, c["n_beams"]) for p, c in zip(pops64, cs)]
    del sts64, pops64, works64
    torch.cuda.empty_cache()
    worst = 0.0
    for (mm, sm), (m6, s6) in zip(mix, f64):
        se = np.sqrt(np.abs(sm) ** 2 + np.abs(s6) ** 2)
        worst = max(worst, float((np.abs(mm - m6) / np.maximum(se, 1e-300)).max()))
    tflops = FLOPS_PER_BEAM_STEP_M24 * N * nsteps / (graph_ms / 1e3) / 1e12
    return {
        "value": N * nsteps / (ms_per_step / 1e3), "unit": "beam-steps/s", "ms_per_step": ms_per_step,
        "steps": steps, "warmup": warmup, "dtype": "f32 trajectories + f64 phase/weights",
        "config": {"workload": name, "system": f"qcle-two-level-{d}d", "instances": len(cs), "n_beams": N,
                   "intervals": nsteps, "dt": dt, "phase_space_dim": m},
        "graph_ms_per_step": graph_ms,
        "launch_shape": {"waves_per_block": cfg[0], "blocks_per_cu": cfg[1], "tiles_per_grab": cfg[2]},
        "autotune_s": t_tune, "autotune_ms": tune_ms,
        "roofline": {"bound": "alu", "kernel": "step_wave_batched<12, 32, float, W>", "achieved": tflops,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": tflops / PEAK_FP32_TFLOPS,
                     "flops_per_unit": FLOPS_PER_BEAM_STEP_M24, "units_per_launch": N * nsteps, "traffic": None,
                     "note": "FP32 stage arithmetic against the FP32 vector peak; time of the whole graph (64 init "
                             "launches, the persistent step, 64 population launches): a lower bound on the "
                             "kernel's rate"},
        "fp64_per_instance": {"value": N * nsteps / (t3 - t2), "ms_per_step": (t3 - t2) * 1e3,
                              "unit": "beam-steps/s"},
        "speedup_vs_fp64_per_instance": (t3 - t2) * 1e3 / ms_per_step,
        "population_diff_over_se": worst,
    }


def run_grad(name, steps, warmup, with_tangent):
    """The derivative workload: the ensemble sampled, stepped with a checkpoint every 100 intervals
    and reduced to populations, then one reverse sweep for the gradient of the upper population in
    (A, B, C, D, p_mean); beside it the plain FP64 forward run (init, step, populations).  For
    d > 1 the timed gradient keeps every interval's stage records in HBM during the forward run
    (shgb_step_recorded, 1648 bytes per beam and interval at d = 12) and the reverse sweep reads
    them; the sweep that runs each segment again from its checkpoint instead is timed beside it."""
    import numpy as np
    import torch
    from paper_1703_06116_amd import shgb, workloads

    c = workloads.config(name)
    N, nsteps, dt, seed, m = c["n_beams"], c["nsteps"], c["dt"], c["seed"], 2 * c["d"]
    every = 100
    kept_mode = m > 2
    mdl = shgb.make_model(c["d"], c["mass"], c["eps"], c["A"], c["B"], c["C"], c["D"], c["lam"], c["bath_omega"])
    spec = shgb.make_init_spec(c["q_mean"], c["q_std"], c["p_dist"], c["p_a"], c["p_b"], c["comp0"])
    dev = "cuda:0"
    st = shgb.State(N, m, device=dev)
    ckpt = torch.empty(max(shgb.checkpoint_bytes(N, m, nsteps, every), 8), dtype=torch.uint8, device=dev)
    adj_work = torch.empty(max(shgb.population_adjoint_workspace(N, m, every), 8), dtype=torch.uint8, device=dev)
    cot = torch.zeros(8, dtype=torch.float64, device=dev)
    cot[0] = 1.0                                       # d Re U_upper
    grad = torch.empty(6, dtype=torch.float64, device=dev)
    pops = torch.empty((4, 5), dtype=torch.float64, device=dev)
    pop_work = torch.empty(max(shgb.populations_workspace(N, m), 8), dtype=torch.uint8, device=dev)
    if kept_mode:
        recs = torch.empty(shgb.record_bytes(N, m, nsteps, every) // 8, dtype=torch.float64, device=dev)
        kwork = torch.empty(max(shgb.population_adjoint_recorded_workspace(N, m, every), 8), dtype=torch.uint8,
                            device=dev)
        grad_k = torch.empty(6, dtype=torch.float64, device=dev)

    def replay_step(evs=None):
        def mark(i):
            if evs is not None:
                evs[i].record()
        mark(0)
        shgb.init_beams(mdl, spec, st, seed)
        shgb.step_checkpointed(mdl, st, nsteps, dt, seed, every=every, ckpt=ckpt)
        shgb.populations(mdl, st, out=pops, work=pop_work)
        mark(1)
        shgb.population_adjoint(mdl, st, ckpt, nsteps, dt, seed, cot, N, every=every, out=grad, work=adj_work)
        mark(2)

    def kept_step(evs=None):
        def mark(i):
            if evs is not None:
                evs[i].record()
        mark(0)
        shgb.init_beams(mdl, spec, st, seed)
        shgb.step_recorded(mdl, st, nsteps, dt, seed, every=every, ckpt=ckpt, recs=recs)
        shgb.populations(mdl, st, out=pops, work=pop_work)
        mark(1)
        shgb.population_adjoint_recorded(mdl, st, ckpt, recs, nsteps, dt, seed, cot, N, every=every, out=grad_k,
                                         work=kwork)
        mark(2)

    def forward_step():
        shgb.init_beams(mdl, spec, st, seed)
        shgb.step_ensemble(mdl, st, nsteps, dt, seed)
        shgb.populations(mdl, st, out=pops, work=pop_work)

    def timed(step):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [[_timer() for _ in range(3)] for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            step(evs[k])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        return (ms, float(np.mean([e[0].elapsed_time(e[1]) for e in evs])),
                float(np.mean([e[1].elapsed_time(e[2]) for e in evs])))

    ms_rep, fwd_rep_ms, rev_rep_ms = timed(replay_step)
    g_rep = grad.cpu().numpy()
    if kept_mode:
        ms_grad, fwd_part_ms, adj_ms = timed(kept_step)
        g = grad_k.cpu().numpy()
        del recs
    else:
        ms_grad, fwd_part_ms, adj_ms, g = ms_rep, fwd_rep_ms, rev_rep_ms, g_rep
    for _ in range(warmup):
        forward_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        forward_step()
    torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t0) * 1e3 / steps
    p = pops.cpu().numpy()
    rev_flops = FLOPS_PER_BEAM_STEP_REV_M24 if kept_mode else FLOPS_PER_BEAM_STEP_ADJ_M24
    tflops = rev_flops * N * nsteps / (adj_ms / 1e3) / 1e12
    line = {
        "value": N * nsteps / (ms_grad / 1e3), "unit": "beam-steps/s", "ms_per_step": ms_grad,
        "steps": steps, "warmup": warmup, "dtype": "f64",
        "config": {"workload": name, "system": f"qcle-two-level-{c['d']}d", "n_beams": N, "intervals": nsteps,
                   "dt": dt, "eps": c["eps"], "phase_space_dim": m, "parameters": 5, "checkpoint_every": every,
                   "stage_records": "kept from the forward run" if kept_mode else "replayed per segment"},
        "note": ("one gradient step = init + forward run (checkpoints every 100 intervals" +
                 (", every interval's stage records kept in HBM" if kept_mode else "") +
                 ") + populations + one reverse sweep for all five parameters; value counts each beam-step "
                 "once"),
        "kernel_ms": {("forward_with_records" if kept_mode else "forward_with_checkpoints"): fwd_part_ms,
                      "reverse_sweep": adj_ms},
        "forward_fp64_ms_per_step": ms_fwd,
        "gradient_over_forward": ms_grad / ms_fwd,
        "replayed_segments": ({"ms_per_step": ms_rep, "gradient_over_forward": ms_rep / ms_fwd,
                               "kernel_ms": {"forward_with_checkpoints": fwd_rep_ms, "reverse_sweep": rev_rep_ms},
                               "max_rel_diff_vs_kept": float(np.abs(g_rep[:5] - g[:5]).max() /
                                                             max(np.abs(g[:5]).max(), 1e-300)),
                               "note": "shgb_step_checkpointed + shgb_population_adjoint: no records kept; "
                                       "the reverse sweep runs each segment again from its checkpoint"}
                              if kept_mode else None),
        "record_bytes": int(shgb.record_bytes(N, m, nsteps, every)) if kept_mode else 0,
        "upper_population": float(p[0, 0] / N),
        "objective_from_reverse_sweep": float(g[5]),
        "d_upper_population": {n: float(g[j]) for j, n in enumerate(("A", "B", "C", "D", "p_mean"))},
        "roofline": {"bound": "alu",
                     "kernel": (f"reverse sweep: aw_reverse_kernel<{c['d']}> over all segments from kept records"
                                if kept_mode else "adjoint_m2_kernel"),
                     "achieved": tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / PEAK_FP64_TFLOPS, "flops_per_unit": rev_flops,
                     "units_per_launch": N * nsteps, "traffic": None,
                     "note": "time of the whole reverse-sweep call (the seed kernel and the reverse kernel): a "
                             "lower bound on the reverse kernel's rate; the split per kernel is in "
                             "profiles/adjoint_wave_qcle12d_grad.md"},
    }
    if with_tangent:
        out = torch.zeros((5, 4, 4), dtype=torch.float64, device=dev)
        work = torch.empty(max(shgb.population_tangent_workspace(N), 8), dtype=torch.uint8, device=dev)
        shgb.init_beams(mdl, spec, st, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        shgb.population_tangent(mdl, st, nsteps, dt, seed, out=out, work=work)
        torch.cuda.synchronize()
        tan_ms = (time.perf_counter() - t0) * 1e3
        o = out.cpu().numpy()
        tan = o[:, 0, 2] / N
        line["tangent_five_directions_ms"] = tan_ms
        line["tangent_over_forward"] = tan_ms / ms_fwd
        line["reverse_vs_tangent_rel"] = float(np.abs(g[:5] - tan).max() / max(np.abs(tan).max(), 1e-300))
    return line


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
    from paper_1703_06116_amd import workloads

    head = a.config or HEADLINE
    extra = [] if (a.config or a.no_extra) else ["qcle12d_2p18", "batch64_d12", "qcle12d_grad"]
    cpu = {}
    if not a.no_cpu_baseline:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(host_cores()) as pool:   # before the GPU is touched
            cpu = cpu_baselines([head] + extra, pool)
            pool.close()
            pool.join()   # every worker has exited before the GPU part starts

    import torch
    torch.cuda.set_device(0)

    def block(name, steps, warmup, headline):
        if name in workloads.BATCH:
            b = run_batch(name, steps, warmup)
        elif name in workloads.GRADIENT:
            b = run_grad(name, steps, warmup, with_tangent=headline)
        else:
            b = run_plain(name, steps, warmup, with_mixed=not a.no_mixed)
        if name in cpu:
            b["cpu_baseline"] = cpu[name]
        torch.cuda.empty_cache()   # the derivative workload keeps 122 GB of records: start it with a clean pool
        return b

    line = block(head, a.steps, a.warmup, headline=True)
    for name in extra:
        line[{"qcle12d_2p18": "c3", "batch64_d12": "c4", "qcle12d_grad": "c5"}[name]] = block(name, 1, 1, False)
    out = {"metric": METRIC, "value": line.pop("value"), "unit": line.pop("unit"), "n_gpus": 1,
           "steps": line.pop("steps"), "warmup": line.pop("warmup"), "ms_per_step": line.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": line.pop("dtype"),
           "data": "synthetic"}
    line["config"]["parallelism"] = "none (1 GPU)"
    out.update(line)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
