"""Test glue shared by the GPU parity tests: build both sides from one config.

Inputs flow one way only: seeded configs and synthetic arrays (workloads) go
to both the oracle and the HIP path; oracle outputs may become HIP inputs;
nothing the HIP path produces is fed to the oracle.
"""

import math

import numpy as np

from oracle import models, sampling, shgb as oshgb
from paper_1703_06116_amd import workloads

RTOL_FP64 = 1e-10   # per-beam state: per beam and field block, error norm / reference norm


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


def field_blocks(s, m):
    """Per-beam blocks of a state given as full matrices (dict of arrays, leading axis = beam):
    name -> (n, k) complex array.  Phase-space coordinates split into the crossing coordinate
    (q1, p1) and the bath (q2.., p2..), the wave vector P into its position and momentum halves,
    Z into its position-position, position-momentum and momentum-momentum blocks."""
    d = m // 2
    X, P, Z = np.asarray(s["X"]), np.asarray(s["P"]), np.asarray(s["Z"])
    n = X.shape[0]
    iu = np.triu_indices(d)
    b = {"q1": X[:, :1], "p1": X[:, d:d + 1], "P_r": P[:, :d], "P_p": P[:, d:],
         "Zrr": Z[:, :d, :d][:, iu[0], iu[1]], "Zrp": Z[:, :d, d:].reshape(n, -1),
         "Zpp": Z[:, d:, d:][:, iu[0], iu[1]]}
    if d > 1:
        b["q_bath"], b["p_bath"] = X[:, 1:d], X[:, d + 1:]
    for f in ("S", "A", "logw", "Lam", "E", "phase"):
        b[f] = np.asarray(s[f]).reshape(n, 1)
    return {k: v.astype(np.complex128) for k, v in b.items()}


# Per-beam relative error of a block is its error norm over max(its reference norm, FLOOR_FRAC x
# the root mean square of that block's norm over the compared beams).  Quantities that pass
# through zero on their way (a wave-vector component, the rate integral Lam just after a hop, the
# phase S of a beam that has only just left a diagonal component) are compared on their own scale
# when they are at least FLOOR_FRAC of the block's typical size and on that scale otherwise; a
# small block is never measured against a large one (bath coordinates against the crossing
# coordinate, as a blockwise maximum over the ensemble would).  FP32 trajectories carry errors
# that are absolute at about 1e-6 of a block's typical size (single-precision increments added to
# the state), so their comparisons take FLOOR_FRAC_MIXED.
FLOOR_FRAC = 1e-2
FLOOR_FRAC_MIXED = 0.1


def compare_states(g, e, rtol=RTOL_FP64, min_ok=0.98, label="", floor_frac=None, max_ties=None):
    """Per-beam comparison of an unpacked GPU state with an oracle ensemble.

    Beams whose oracle run met a threshold or destination tie are excluded
    (and counted): at most max_ties of them when it is given (the callers set
    it from the count the oracle run meets plus a margin), else at most the
    fraction 1 - min_ok.  All others must have identical hop counts and
    components, and for every beam and every field block (field_blocks) the
    error norm over the reference norm must be at most rtol.  Returns the
    worst per-beam relative error of each block and the number of excluded
    beams.
    """
    ok = (e.thr_ties == 0) & (e.dest_ties == 0)
    if max_ties is not None:
        assert int((~ok).sum()) <= max_ties, f"{label}: too many ties {int((~ok).sum())} > {max_ties}"
    else:
        assert ok.mean() >= min_ok, f"{label}: too many ties {int((~ok).sum())}"
    bad = np.flatnonzero(ok & ((g["nhop"] != e.nhop) | (g["comp"] != e.comp)))
    if bad.size:
        lines = [f"{label}: {bad.size} beams differ in hops/components; first ones:"]
        for b in bad[:8]:
            lines.append(f"  beam {b}: gpu comp {g['comp'][b]} nhop {g['nhop'][b]} phase {g['phase'][b]} "
                         f"logw {g['logw'][b]:.6f} | oracle comp {e.comp[b]} nhop {e.nhop[b]} "
                         f"phase {e.phase[b]} logw {e.logw[b]:.6f} log {e.hop_log[b]}")
        raise AssertionError("\n".join(lines))
    if floor_frac is None:
        floor_frac = FLOOR_FRAC if rtol < 1e-6 else FLOOR_FRAC_MIXED
    m = e.X.shape[1]
    ref = field_blocks(dict(X=e.X, P=e.P, Z=e.M + 1j * e.N, S=e.S, A=e.A, logw=e.logw, Lam=e.Lam, E=e.E,
                            phase=e.phase), m)
    got = field_blocks(g, m)
    errs, worst_beam = {}, {}
    for k in ref:
        r, x = ref[k][ok], got[k][ok]
        if r.shape[0] == 0:
            errs[k] = 0.0
            continue
        rn = np.linalg.norm(r, axis=1)
        floor = floor_frac * math.sqrt(float(np.mean(rn * rn)))
        den = np.maximum(rn, floor)
        en = np.linalg.norm(x - r, axis=1)
        rel = np.where(den > 0, en / np.where(den > 0, den, 1.0), en)
        errs[k] = float(rel.max())
        w = int(rel.argmax())
        worst_beam[k] = (int(np.flatnonzero(ok)[w]), float(rn[w]), floor)
    bad = {k: (v, worst_beam.get(k)) for k, v in errs.items() if not (v <= rtol)}
    assert not bad, f"{label}: per-beam blocks beyond {rtol} (error, (beam, its norm, floor)): {bad}; all: {errs}"
    return errs, int((~ok).sum())
