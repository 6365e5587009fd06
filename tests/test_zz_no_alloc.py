"""The allocation-free entry point p3t_compute_cutoffs_noalloc (through the
C ABI) against the entry point it varies, p3t_compute_cutoffs: the same
radii bit for bit (the same passes, with the per-particle terms recomputed
instead of kept), and the oracle's to 1e-12.  Two calls in a row, the second
on a smaller input, so that the shared device scratch left by the first call
cannot leak into the second; the shared mode; and an input beyond the
scratch limit, rejected before any launch."""
import numpy as np
import pytest
import torch

import diskgen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def params(gpu, p, **kw):
    return gpu.Params.defaults().replace(
        G=p.G, m_star=p.m_star, r_cut0=p.r_cut0, r_cut1=p.r_cut1, r_search0=p.r_search0, r_search1=p.r_search1,
        dt_soft=p.dt_soft, hill_length=p.hill_length, vran_bins=p.vran_bins, vran_min_count=p.vran_min_count,
        cutoff_mode=p.cutoff_mode, **kw)


@pytest.mark.parametrize("mode", [0, 1], ids=["individual", "shared"])
def test_noalloc_cutoffs_equal_the_context_entry_point(gpu, orc, mode):
    p = orc.Params(cutoff_mode=mode)
    gp = params(gpu, p)
    ctx = gpu.Context(gp)
    for d in (diskgen.workload("disk64k_masslaw"), diskgen.make_disk(3000, 0.9, 1.1, seed=8)):
        pos, vel, m = T(d.pos), T(d.vel), T(d.mass)
        ref = ctx.compute_cutoffs(pos, vel, m)
        out = tuple(torch.full((d.n,), float("nan"), dtype=torch.float64, device=DEV) for _ in range(3))
        gpu.compute_cutoffs_noalloc(gp, pos, vel, m, out)
        torch.cuda.synchronize()
        for a, b, name in zip(out, ref, ("r_out", "r_search", "v_ran")):
            assert torch.equal(a, b), (d.n, name)
        ro, rs, vr = orc.cutoffs(d.pos, d.vel, d.mass, p)
        for a, b in zip(out, (ro, rs, vr)):
            assert np.allclose(a.cpu().numpy(), b, rtol=1e-12, atol=0)
        print("n", d.n, "mode", mode, "r_out median", float(out[0].median()))


def test_noalloc_rejects_inputs_beyond_its_scratch(gpu, orc):
    """2^21 + 4096 particles with 256 bins need more than the 8 MiB: the call
    returns P3T_ERR_CAPACITY and leaves the outputs untouched."""
    n = (1 << 21) + 4096
    gp = params(gpu, orc.Params(vran_bins=256))
    pos = torch.ones((3, n), dtype=torch.float64, device=DEV)
    vel = torch.ones((3, n), dtype=torch.float64, device=DEV)
    m = torch.ones(n, dtype=torch.float64, device=DEV)
    out = tuple(torch.zeros(n, dtype=torch.float64, device=DEV) for _ in range(3))
    with pytest.raises(gpu.P3TError) as ei:
        gpu.compute_cutoffs_noalloc(gp, pos, vel, m, out)
    assert ei.value.status == 2 and "8388608" in str(ei.value)
    torch.cuda.synchronize()
    assert all(int(torch.count_nonzero(t)) == 0 for t in out)
