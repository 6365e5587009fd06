"""Perfect-accretion collisions (Section 2.5.1) on the GPU against the
oracle: the collision integrator on caller-given clusters (mergers, the
composite map, states, dissipation sums, energy bookkeeping), the merge
compaction bit for bit, the no-collision limit, and the full step driver
with mergers against the oracle step.

Mergers are discrete decisions taken on FP64 predicted states on both
sides; like the block-step sequence (see the Hermite parity test) a
rounding-level difference can flip one inside a compacted cluster.  Clusters
with the same block-step count, merger count and composite map are compared
up to rounding; the others are counted and must stay few.
"""
import math

import numpy as np
import pytest
import torch

import diskgen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def gparams(gpu, p, **kw):
    return gpu.Params.defaults().replace(G=p.G, m_star=p.m_star, gamma=p.gamma, r_cut0=p.r_cut0, r_cut1=p.r_cut1,
                                         r_search0=p.r_search0, r_search1=p.r_search1, r_search2=p.r_search2,
                                         r_search3=p.r_search3, dt_soft=p.dt_soft, eta=p.eta, eta0=p.eta0,
                                         k_max=p.k_max, **kw)


def clusters(orc, n_clusters, n_max, compact, eta=0.02, seed=4):
    p = orc.Params(eta=eta, eta0=0.1 * eta)
    d = diskgen.workload("disk64k_masslaw")
    ro, _, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
    cl = diskgen.hermite_clusters(d, n_clusters=n_clusters, seed=seed, n_max=n_max, r_out=ro, compact=compact)
    return p, cl


@pytest.mark.parametrize("n_max", [8, 64])
def test_hermite_collide_matches_oracle(gpu, orc, n_max):
    rho = orc.density_code(2.0)
    f = 200.0
    p, cl = clusters(orc, 3000, n_max, 0.7)
    mem = np.arange(cl["pos"].shape[1], dtype=np.int32)
    ro_ = orc.hermite_collide(cl["pos"], cl["vel"], cl["mass"], cl["r_out"], cl["cl_ptr"], mem, p, f, rho)
    assert ro_["status"] == 0
    ctx = gpu.Context(gparams(gpu, p))
    pos, vel = T(cl["pos"]), T(cl["vel"])
    out = ctx.hermite_collide(pos, vel, T(cl["mass"]), T(cl["r_out"]), T(cl["cl_ptr"], torch.int32),
                              T(mem, torch.int32), f, rho, steps=True)
    from paper_2007_15432_amd import _lib

    assert ctx.status() & _lib.FLAG_COLL_UNCHECKED == 0
    xg, vg = pos.cpu().numpy(), vel.cpu().numpy()
    mg = out["merged_into"].cpu().numpy()
    eg = out["eps"].cpu().numpy()
    ng = out["nsteps"].cpu().numpy()
    relg = out["e_rel"].cpu().numpy()
    ptr = cl["cl_ptr"]
    nc = len(ptr) - 1
    # collisions per cluster on the GPU: the composites in the map
    ncg = np.array([len(np.unique(mg[a:b])) for a, b in zip(ptr[:-1], ptr[1:])])
    nco = np.array([len(np.unique(ro_["merged_into"][a:b])) for a, b in zip(ptr[:-1], ptr[1:])])
    same = (ng == ro_["nsteps"]) & (ncg == nco)
    same &= np.array([np.array_equal(mg[a:b], ro_["merged_into"][a:b]) for a, b in zip(ptr[:-1], ptr[1:])])
    hit = ro_["ncoll"] > 0
    print(f"n_max {n_max}: clusters {nc}, with mergers {hit.sum()}, mergers oracle {ro_['ncoll'].sum()} "
          f"gpu {out['ncoll']}, same path {same.sum()} ({same[hit].sum()} of those with mergers)")
    assert hit.sum() >= 100
    assert same.mean() >= 0.97 and same[hit].mean() >= 0.9
    # every merger removes one composite
    assert out["ncoll"] == int(((ptr[1:] - ptr[:-1]) - ncg).sum())
    assert np.array_equal(ro_["ncoll"], (ptr[1:] - ptr[:-1]) - nco)
    dx = np.array([np.abs(xg[:, a:b] - ro_["pos"][:, a:b]).max() for a, b in zip(ptr[:-1], ptr[1:])])
    print("max |dx| same path", dx[same].max(), "median", np.median(dx[same]))
    assert np.median(dx[same]) < 1e-13 and np.mean(dx[same] < 1e-10) >= 0.97 and dx[same].max() < 1e-5
    # dissipation sums: up to rounding on the same path
    scale = np.abs(ro_["eps"]).max(axis=1, keepdims=True) + 1e-300
    de = (np.abs(eg - ro_["eps"]) / scale)[same & hit]
    print("eps relative difference (same path): median", np.median(de), "max", de.max())
    assert np.median(de) < 1e-10 and np.mean(de.max(axis=1) < 1e-6) >= 0.97
    # energy bookkeeping: the GPU's |E_end + eps5 - E_start| / |E_start| against the oracle's
    rel_o = np.abs(ro_["e1"] + ro_["eps"][:, 5] - ro_["e0"]) / np.abs(ro_["e0"])
    ok = np.abs(relg - rel_o) <= np.maximum(0.05 * rel_o, 1e-13)
    print("bookkeeping within 5%:", int(ok[same].sum()), "of", int(same.sum()), "worst gpu", relg.max(),
          "oracle", rel_o.max())
    assert ok[same].mean() >= 0.97 and relg.max() <= 10 * rel_o.max() + 1e-12


def test_no_collision_limit_is_the_hermite_path(gpu, orc):
    """f = 0: no merger, and the collision kernel (every cluster of 2..64 on
    the wavefront path) reproduces the plain path up to rounding."""
    p, cl = clusters(orc, 2000, 48, None)  # natural clusters: no close encounter runs into the step limit
    mem = T(np.arange(cl["pos"].shape[1], dtype=np.int32), torch.int32)
    ctx = gpu.Context(gparams(gpu, p))
    ptr = T(cl["cl_ptr"], torch.int32)
    p1, v1 = T(cl["pos"]), T(cl["vel"])
    _, ns1 = ctx.hermite_cluster_step(p1, v1, T(cl["mass"]), T(cl["r_out"]), ptr, mem, steps=True)
    p2, v2 = T(cl["pos"]), T(cl["vel"])
    out = ctx.hermite_collide(p2, v2, T(cl["mass"]), T(cl["r_out"]), ptr, mem, 0.0, 1.0, steps=True)
    assert out["ncoll"] == 0 and torch.equal(out["merged_into"], mem) and bool((out["eps"] == 0).all())
    same = (ns1 == out["nsteps"]).cpu().numpy()
    dx = (p1 - p2).abs().amax(0).cpu().numpy()
    print("same steps", same.mean(), "max |dx|", dx.max())
    assert same.mean() >= 0.97


def test_merge_bodies_matches_oracle(gpu, orc):
    from oracle import step as ostep

    rng = np.random.default_rng(7)
    n = 100_000
    pos, vel = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    mass = rng.uniform(1e-10, 1e-9, n)
    dt_hard = rng.uniform(0, 1, n)
    steps = rng.integers(1, 1000, n).astype(np.int32)
    merged = np.arange(n, dtype=np.int32)
    # composites of 2..4 consecutive-ish indices, the lowest index the survivor
    heads = np.sort(rng.choice(n - 10, 3000, replace=False))
    heads = heads[np.concatenate([[True], np.diff(heads) > 8])]
    for h in heads:
        k = rng.integers(1, 4)
        parts = h + np.sort(rng.choice(np.arange(1, 8), k, replace=False))
        merged[parts] = h
        pos[:, parts] = pos[:, [h]]
        vel[:, parts] = vel[:, [h]]
    ro = ostep.merge_bodies(pos, vel, mass, dt_hard, merged)
    ctx = gpu.Context(gpu.Params.defaults())
    gp, gv, gm, gd, gs = T(pos), T(vel), T(mass), T(dt_hard), T(steps, torch.int32)
    nn = ctx.merge_bodies(T(merged, torch.int32), gp, gv, gm, dt_hard=gd, steps=gs)
    keep = ro[4]
    assert nn == int(keep.sum())
    assert np.array_equal(gp.view(-1)[:3 * nn].view(3, nn).cpu().numpy(), ro[0])
    assert np.array_equal(gv.view(-1)[:3 * nn].view(3, nn).cpu().numpy(), ro[1])
    assert np.array_equal(gm[:nn].cpu().numpy(), ro[2])
    assert np.array_equal(gd[:nn].cpu().numpy(), ro[3])
    assert np.array_equal(gs[:nn].cpu().numpy(), steps[keep])
    # a map that does not name composites is refused before anything moves
    bad = merged.copy()
    bad[5] = 7  # points above itself
    before = gm.clone()
    with pytest.raises(gpu.P3TError) as e:
        ctx.merge_bodies(T(bad, torch.int32), T(pos), T(vel), gm)
    assert e.value.status == 1
    assert torch.equal(gm, before)


def test_driver_with_collisions_matches_oracle_step(gpu, orc):
    """The serial step driver with perfect accretion on a dense ring against
    the oracle step: the same mergers step by step (particle count, total
    mass), states up to rounding, and the Newtonian energy with the booked
    dissipation (eps with W = 1) nearly conserved."""
    from oracle import step as ostep
    from paper_2007_15432_amd.driver import P3TStepper

    rho = orc.density_code(2.0)
    f = 150.0
    d = diskgen.dense_ring(1024, seed=11)
    p = orc.Params(dt_soft=1.0 / 64)
    ro, rs, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
    s = ostep.init(d.pos, d.vel, d.mass, ro, rs, p)
    mo, r_o, r_s = d.mass.copy(), ro, rs
    ctx = gpu.Context(gparams(gpu, p, theta=0.0, isolated=1))
    st = P3TStepper(ctx, T(d.pos), T(d.vel), T(d.mass), collisions=(f, rho))
    e_start = ostep.total_energy(d.pos, d.vel, d.mass, p)
    eps_o = np.zeros(6)
    for k in range(4):
        s, mo, r_o, r_s, eps, removed = ostep.step_collide(s, mo, r_o, r_s, p, f, rho)
        eps_o += eps
        st.step()
        ng = st.n
        print(f"step {k}: oracle n {mo.shape[0]} (removed {removed}), gpu n {ng}, mergers gpu {st.n_collisions}")
        assert ng == mo.shape[0]
        assert np.array_equal(st.mass.cpu().numpy(), mo)
        dx = np.abs(st.pos.cpu().numpy() - s.pos).max()
        print("   max |dx|", dx)
        assert dx < 1e-9
    e_end = ostep.total_energy(st.pos.cpu().numpy(), st.vel.cpu().numpy(), st.mass.cpu().numpy(), p)
    book = (e_end + st.eps[4] - e_start) / abs(e_start)
    raw = (e_end - e_start) / abs(e_start)
    print("energy change", raw, "with the booked dissipation", book, "eps gpu", st.eps, "oracle", eps_o)
    assert abs(book) < 1e-2 * abs(raw)
    de = np.abs(np.array(st.eps) - eps_o)
    print("eps |gpu - oracle| / max|eps|:", de / np.abs(eps_o).max(), "relative:", de / np.abs(eps_o))
    # eps_2 and eps_3 are differences of potentials that cancel: a rounding-level absolute bar
    assert np.all(de <= 1e-8 * np.abs(eps_o) + 1e-9 * np.abs(eps_o).max())
