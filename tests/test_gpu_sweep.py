"""The cut-off schemes of Section 3.2.2 on the GPU path: the average number
of neighbours <n_b> and the largest neighbour cluster n_b,max as functions
of Rcut0 (theta = 0.5, dt = 1/64) on the 65,536-particle mass-law disk.

Under the shared cut-off (eq. (rout1)) every pair uses the largest radius,
which the most massive particles set, so <n_b> grows steeply with Rcut0
(the paper: roughly as Rcut0^3; on this disk, thinner than the search radii,
the neighbours fill a layer and the growth is close to Rcut0^2) and the
clusters percolate; under the individual cut-off (eq. (rout2)) <n_b> stays
several times smaller and the clusters small.  Each point is checked
against the oracle's neighbour rows on a sample of particles.
"""
import numpy as np
import pytest
import torch

import diskgen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

SCHEMES = {"shared": dict(cutoff_mode=1), "individual": dict(cutoff_mode=0, r_cut1=0.0, r_search1=0.0),
           "individual_vran": dict(cutoff_mode=0)}


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def sweep(gpu, orc):
    d = diskgen.workload("disk64k_masslaw")
    pos, vel, m = T(d.pos), T(d.vel), T(d.mass)
    idx = diskgen.sample_indices(d.n, 512, 77)
    out = {}
    for name, kw in SCHEMES.items():
        for rc in (1.0, 2.0, 4.0, 8.0):
            p = orc.Params(r_cut0=rc, dt_soft=1.0 / 64, **{k: v for k, v in kw.items()})
            gp = gpu.Params.defaults().replace(theta=0.5, multipole=2, dt_soft=p.dt_soft, r_cut0=rc, **kw)
            ctx = gpu.Context(gp)
            ro, rs, _ = ctx.compute_cutoffs(pos, vel, m)
            ctx.evaluate(pos, vel, m, ro, rs, graph=False)
            rp, col, lab = ctx.neighbour_list(labels=True)
            rp = rp.cpu().numpy()
            # the sampled rows against the oracle's, on the oracle's radii
            ro_o, rs_o, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
            assert np.allclose(ro.cpu().numpy(), ro_o, rtol=1e-12)
            rp_o, col_o = orc.neighbour_rows(d.pos, d.vel, d.mass, ro.cpu().numpy(), rs.cpu().numpy(), p, idx=idx)
            assert np.array_equal(np.diff(rp)[idx], np.diff(rp_o))
            out[(name, rc)] = (rp[-1] / d.n, int(torch.bincount(lab.long()).max()))
            print(name, rc, "mean neighbours", out[(name, rc)][0], "largest cluster", out[(name, rc)][1])
    return d.n, out


def test_shared_cutoff_neighbours_grow_steeply_and_percolate(sweep):
    n, out = sweep
    nb = np.array([out[("shared", rc)][0] for rc in (1.0, 2.0, 4.0, 8.0)])
    slope = np.polyfit(np.log([1.0, 2.0, 4.0, 8.0]), np.log(nb), 1)[0]
    print("shared: <n_b> slope in Rcut0", slope)
    assert 1.8 < slope < 3.2
    assert out[("shared", 8.0)][1] > n // 2  # percolated


def test_individual_cutoff_keeps_clusters_small(sweep):
    n, out = sweep
    for name in ("individual", "individual_vran"):
        for rc in (1.0, 2.0, 4.0, 8.0):
            nb, largest = out[(name, rc)]
            assert nb <= 0.2 * out[("shared", rc)][0]
            assert largest < 100
