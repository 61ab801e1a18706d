"""Test glue shared by the GPU parity tests: build both sides from one config.

Inputs flow one way only: seeded configs and synthetic arrays (workloads) go
to both the oracle and the HIP path; oracle outputs may become HIP inputs;
nothing the HIP path produces is fed to the oracle.
"""

import numpy as np

from oracle import models, sampling, shgb as oshgb
from paper_1703_06116_amd import workloads

RTOL_FP64 = 1e-10   # per-beam state, blockwise relative (max-abs error / max-abs reference)


def oracle_model(c):
    return models.QCLE(c["A"], c["B"], c["C"], c["D"], c["mass"], d=c["d"], lam=c.get("lam", 0.0),
                       bath_omega=c["bath_omega"])


def gpu_model(c):
    from paper_1703_06116_amd import shgb
    return shgb.make_model(c["d"], c["mass"], c["eps"], c["A"], c["B"], c["C"], c["D"],
                           c.get("lam", 0.0), c["bath_omega"])


def gpu_spec(c):
    from paper_1703_06116_amd import shgb
    return shgb.make_init_spec(c["q_mean"], c["q_std"], c["p_dist"], c["p_a"], c["p_b"], c["comp0"])


def oracle_init(c, n, offset=0):
    return sampling.init_beams(oracle_model(c), n, c["eps"], c["seed"], c["q_mean"], c["q_std"],
                               c["p_dist"], c["p_a"], c["p_b"], c["comp0"], beam_id_offset=offset)


def oracle_init_ids(c, ids):
    """Oracle initial beams for arbitrary global ids (each sampled on its own)."""
    parts = [oracle_init(c, 1, int(g)) for g in ids]
    e = oshgb.Ensemble(len(ids), parts[0].m, parts[0].n_comp)
    for f in ("X", "P", "M", "N", "S", "A", "logw", "phase", "Lam", "E", "comp", "nhop", "gid"):
        getattr(e, f)[:] = np.concatenate([getattr(p, f) for p in parts])
    return e


def ensemble_from_arrays(a, n_comp=4, gid0=0):
    """Oracle ensemble from host arrays (workloads.synthetic_ensemble or an oracle dump)."""
    X = np.asarray(a["X"])
    n, m = X.shape
    e = oshgb.Ensemble(n, m, n_comp)
    e.X[:] = X
    e.P[:] = a["P"]
    e.M[:] = np.real(a["Z"])
    e.N[:] = np.imag(a["Z"])
    e.S[:] = a["S"]
    e.A[:] = a["A"]
    e.logw[:] = a["logw"]
    e.phase[:] = a["phase"]
    e.Lam[:] = a["Lam"]
    e.E[:] = a["E"]
    e.comp[:] = a["comp"]
    e.nhop[:] = a["nhop"]
    e.gid[:] = gid0 + np.arange(n, dtype=np.uint64)
    return e


def arrays_from_ensemble(e):
    return dict(X=e.X, P=e.P, Z=e.M + 1j * e.N, S=e.S, A=e.A, logw=e.logw, phase=e.phase, Lam=e.Lam,
                E=e.E, comp=e.comp, nhop=e.nhop)


def blockrel(a, b):
    ref = np.abs(b).max()
    return np.abs(a - b).max() / max(ref, 1e-300)


def compare_states(g, e, rtol=RTOL_FP64, min_ok=0.98, label=""):
    """Per-beam comparison of an unpacked GPU state with an oracle ensemble.

    Beams whose oracle run met a threshold or destination tie are excluded
    (and counted); all others must have identical hop counts and components
    and agree blockwise to rtol in every continuous field.
    """
    ok = (e.thr_ties == 0) & (e.dest_ties == 0)
    assert ok.mean() >= min_ok, f"{label}: too many ties {int((~ok).sum())}"
    bad = np.flatnonzero(ok & ((g["nhop"] != e.nhop) | (g["comp"] != e.comp)))
    if bad.size:
        lines = [f"{label}: {bad.size} beams differ in hops/components; first ones:"]
        for b in bad[:8]:
            lines.append(f"  beam {b}: gpu comp {g['comp'][b]} nhop {g['nhop'][b]} phase {g['phase'][b]} "
                         f"logw {g['logw'][b]:.6f} | oracle comp {e.comp[b]} nhop {e.nhop[b]} "
                         f"phase {e.phase[b]} logw {e.logw[b]:.6f} log {e.hop_log[b]}")
        raise AssertionError("\n".join(lines))
    errs = {
        "X": blockrel(g["X"][ok], e.X[ok]),
        "P": blockrel(g["P"][ok], e.P[ok]) if np.abs(e.P[ok]).max() > 0 else np.abs(g["P"][ok]).max(),
        "Z": blockrel(g["Z"][ok], (e.M + 1j * e.N)[ok]),
        "S": blockrel(g["S"][ok], e.S[ok]) if np.abs(e.S[ok]).max() > 0 else np.abs(g["S"][ok]).max(),
        "Lam": blockrel(g["Lam"][ok], e.Lam[ok]) if np.abs(e.Lam[ok]).max() > 0 else 0.0,
        "logw": blockrel(g["logw"][ok], e.logw[ok]) if np.abs(e.logw[ok]).max() > 0 else 0.0,
        "A": blockrel(g["A"][ok], e.A[ok]),
        "E": blockrel(g["E"][ok], e.E[ok]),
        "phase": np.abs(g["phase"][ok] - e.phase[ok]).max(),
    }
    m = e.X.shape[1]
    if m > 2:   # per block of Z, for the message
        d = m // 2
        Zg, Ze = g["Z"][ok], (e.M + 1j * e.N)[ok]
        for name, sl in (("Zrr", (slice(0, d), slice(0, d))), ("Zrp", (slice(0, d), slice(d, m))),
                         ("Zpp", (slice(d, m), slice(d, m)))):
            errs[name + "_abs"] = float(np.abs(Zg[:, sl[0], sl[1]] - Ze[:, sl[0], sl[1]]).max())
            errs[name + "_max"] = float(np.abs(Ze[:, sl[0], sl[1]]).max())
    bad = {k: v for k, v in errs.items() if not k.endswith(("_abs", "_max")) and not (v <= rtol)}
    assert not bad, f"{label}: fields beyond {rtol}: {bad}; all: {errs}"
    return errs, int((~ok).sum())
