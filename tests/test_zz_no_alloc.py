"""The allocation-free populations entry point (shgb_populations_noalloc):
its partial sums live in the library's own device array instead of a caller
workspace.  Its output must equal shgb_populations' bitwise, call after call,
also when a call follows one with a larger ensemble (so stale partials of the
earlier call sit beyond the blocks the later call uses)."""

import numpy as np
import pytest
import torch

from paper_1703_06116_amd import workloads

from _parity import gpu_model

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,sizes", [(2, (300_000, 70_001)), (24, (5000, 37)), (4, (4097, 1))])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_populations_equal_workspace_populations(gpu, m, sizes, precision):
    d = m // 2
    c = workloads.config("qcle12d_2p18" if d > 1 else "qcle1d_1e6", d=d, bath_omega=workloads.bath_omega(d))
    mdl = gpu_model(c)
    for call, n in enumerate(sizes):
        a = workloads.synthetic_ensemble(n, m, seed=100 + call, a0=(2 * np.pi * c["eps"]) ** (-d))
        st = gpu.pack(a, precision=precision)
        ref = gpu.populations(mdl, st)
        out = torch.full((4, 5), float("nan"), dtype=torch.float64, device="cuda")
        diag, diag_ref = gpu.new_diag(), gpu.new_diag()
        gpu.populations(mdl, st, out=ref, diag=diag_ref)
        gpu.populations_noalloc(mdl, st, out, diag=diag)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (m, n, precision, (out - ref).abs().max().item())
        assert torch.equal(diag, diag_ref)
        assert out[:, 4].sum().item() == n


def test_noalloc_rejects_bad_arguments(gpu):
    c = workloads.config("qcle1d_1e4")
    st = gpu.State(10, 2)
    assert gpu._lib.shgb_populations_noalloc(None, None, None, None, None) == -1   # SHGB_EINVAL
    out = torch.empty((4, 5), dtype=torch.float64, device="cuda")
    bad = gpu_model(dict(c, d=3, bath_omega=workloads.bath_omega(3)))    # m = 6 model, m = 2 state
    with pytest.raises(gpu.ShgbError):
        gpu.populations_noalloc(bad, st, out)
