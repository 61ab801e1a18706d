"""Results do not depend on the leading dimension of the state.

A state may be a window of a wider allocation: row f of beam b sits at
f * ld + b.  With ld chosen so that the offsets of the last rows pass 2^31
elements, every entry point must give bitwise the results of the same beams
stored with ld = n, which holds only if each kernel forms its row offsets in
64-bit arithmetic.  Each wide state takes 11-38 GB of device memory.
"""

import numpy as np
import pytest
import torch

from paper_1703_06116_amd import workloads

from _parity import gpu_model, gpu_spec

pytestmark = pytest.mark.gpu


def _config(m, n):
    # beams start near the avoided crossing so that they hop within the run
    if m == 2:
        return workloads.config("qcle1d_1e4", n_beams=n, q_mean=-2.5, q_std=0.3, p_a=30.0)
    return workloads.config("qcle12d_2p18", d=12, bath_omega=workloads.bath_omega(12), n_beams=n,
                            q_mean=-2.5, q_std=0.3, p_a=30.0)


def _run(gpu, c, m, ld, precision, nsteps, batched=False):
    n = c["n_beams"]
    mdl = gpu_model(c)
    st = gpu.State(n, m, ld=ld, beam_id_offset=777, precision=precision)
    gpu.init_beams(mdl, gpu_spec(c), st, c["seed"])
    diag = gpu.new_diag()
    if batched:   # the persistent batched kernel on a one-instance batch
        gpu.Batch([mdl], [st], [c["seed"]]).step(nsteps, c["dt"], diag=diag)
    else:
        gpu.step_ensemble(mdl, st, nsteps, c["dt"], c["seed"], diag=diag)
    gpu.hop(mdl, st, torch.arange(0, n, 5, dtype=torch.int32, device="cuda"), c["seed"] + 1, diag=diag)
    out = {"state": gpu.unpack(st), "pop": gpu.populations(mdl, st, diag=diag).cpu().numpy()}
    pts = workloads.points_near(out["state"]["X"], c["eps"], 300, seed=5)
    out["field"] = gpu.reconstruct(mdl, st, torch.from_numpy(pts).cuda()).cpu().numpy()
    if precision == "fp64":
        out["tangent"] = gpu.population_tangent(mdl, st, 40, c["dt"], c["seed"], dirs=[1, 4], diag=diag)
        out["tangent"] = out["tangent"].cpu().numpy()
    out["diag"] = diag.cpu().numpy()
    del st
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


# (m, n, ld, intervals): the last trajectory rows start beyond 2^31 elements
# in both precisions (m = 2: row 9 of the 10 trajectory rows at ld = 2.5e8;
# m = 24: rows 512 to 647 at ld = 2^22 + 5).
CASES = [(2, 1000 + 37, 250_000_000, 400), (24, 3 * 64 + 9, (1 << 22) + 5, 400)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("m,n,ld,nsteps", CASES)
def test_results_do_not_depend_on_ld_past_2_31(gpu, m, n, ld, nsteps, precision):
    traj_rows = 2 * m + m * (m + 1)
    assert (traj_rows - 1) * ld > 2**31
    c = _config(m, n)
    print(f"m={m} n={n} ld={ld} precision={precision}", flush=True)
    ref = _run(gpu, c, m, None, precision, nsteps)
    assert ref["diag"][0] > 0                      # hops happened
    for batched in (False, True):
        wide = _run(gpu, c, m, ld, precision, nsteps, batched)
        for k, v in ref["state"].items():
            np.testing.assert_array_equal(wide["state"][k], v, err_msg=f"{k} batched={batched}")
        for k in ("pop", "field", "tangent", "diag"):
            if k in ref:
                np.testing.assert_array_equal(wide[k], ref[k], err_msg=f"{k} batched={batched}")
