"""Pins of the oracle's perfect-accretion collisions (Section 2.5.1) against
facts that do not come from the oracle itself:

* with f = 0 nothing collides and the collision integrator is the plain
  Hermite integrator, bit for bit;
* the radial infall of two bodies from rest (star switched off): the
  merger's time brackets the analytic contact time of the two-body radial
  orbit, the merged body keeps the centre of mass and the momentum, and the
  Newtonian energy released (eps with W replaced by one) is the energy of
  the initial state, -G m^2 / d;
* the bookkeeping identities: (W = 1 sum) - (1 - W sum) = eps1 + eps3, and
  E_hard(end) + sum eps5 = E_hard(start) up to the integration error on
  compacted disk clusters with many mergers;
* after a merger at the first block step the composite follows the orbit
  of one body of the combined mass (plain Hermite run on the merged system).
"""
import math

import numpy as np
import pytest

import diskgen
import oracle

RHO = oracle.density_code(2.0)  # 2 g / cm^3 (Section 3.1)


def radius(m):
    return (3.0 * m / (4.0 * math.pi * RHO)) ** (1.0 / 3.0)


def one_cluster(n):
    return np.array([0, n], dtype=np.int32), np.arange(n, dtype=np.int32)


def test_no_collision_is_plain_hermite():
    p = oracle.Params(eta=0.02, eta0=0.002)
    d = diskgen.workload("disk64k_masslaw")
    ro, _, _ = oracle.cutoffs(d.pos, d.vel, d.mass, p)
    cl = diskgen.hermite_clusters(d, n_clusters=300, seed=4, n_max=24, r_out=ro, compact=0.7)
    mem = np.arange(cl["pos"].shape[1], dtype=np.int32)
    x, v, e0, e1, ns, st = oracle.hermite_clusters(cl["pos"], cl["vel"], cl["mass"], cl["r_out"], cl["cl_ptr"], mem,
                                                   p)
    r = oracle.hermite_collide(cl["pos"], cl["vel"], cl["mass"], cl["r_out"], cl["cl_ptr"], mem, p, 0.0, RHO)
    assert st == r["status"] == 0
    assert np.array_equal(x, r["pos"]) and np.array_equal(v, r["vel"])
    assert np.array_equal(e0, r["e0"]) and np.array_equal(e1, r["e1"]) and np.array_equal(ns, r["nsteps"])
    assert np.all(r["ncoll"] == 0) and np.array_equal(r["merged_into"], mem) and np.all(r["eps"] == 0.0)


@pytest.mark.parametrize("f", [1.0, 3.0])
def test_radial_infall(f):
    m, d = 1e-9, 1e-4
    p = oracle.Params(m_star=1e-30, eta=1e-3, eta0=1e-4, dt_soft=0.05)
    pos = np.array([[1 - d / 2, 1 + d / 2], [0.0, 0.0], [0.0, 0.0]])
    vel = np.array([[0.0, 0.0], [1e-3, 1e-3], [0.0, 0.0]])  # common drift, no relative motion
    mass = np.array([m, 2 * m])
    ro = np.full(2, 10 * d)
    dh = np.full(2, 1e-5)
    r = oracle.hermite_collide(pos, vel, mass, ro, *one_cluster(2), p, f, RHO, dt_hard=dh)
    assert r["status"] == 0 and r["ncoll"][0] == 1
    M = 3 * m
    s = f * (radius(m) + radius(2 * m))
    tff = math.sqrt(d ** 3 / (2 * M))
    tc = tff * (math.sqrt((s / d) * (1 - s / d)) + math.acos(math.sqrt(s / d)))
    t = r["tcoll"][0] * p.dt_soft * 2.0 ** -40
    dyn = math.sqrt(s ** 3 / M)  # dynamical time at contact: the steps there are a small fraction of it
    print(f"f {f}: merger at {t:.9f}, analytic contact {tc:.9f}, dynamical time there {dyn:.2e}")
    assert tc - 1e-9 <= t <= tc + dyn
    # the merged body: centre of mass and momentum (both parts carry the state)
    assert np.array_equal(r["merged_into"], [0, 0])
    assert np.array_equal(r["pos"][:, 0], r["pos"][:, 1]) and np.array_equal(r["vel"][:, 0], r["vel"][:, 1])
    p_tot = mass[0] * vel[:, 0] + mass[1] * vel[:, 1]
    assert np.allclose(M * r["vel"][:, 0], p_tot, rtol=0, atol=1e-15 * M)
    x_com = (mass[0] * pos[:, 0] + mass[1] * pos[:, 1]) / M + 0.05 * np.array([0.0, 1e-3, 0.0])
    assert np.allclose(r["pos"][:, 0], x_com, rtol=0, atol=1e-13)
    # energy released = Newtonian energy of the initial state (the merged body rests in the COM frame)
    e_init = -m * 2 * m / d
    eps = r["eps"][0]
    print("eps", eps, "initial Newtonian energy", e_init)
    assert abs(eps[4] - e_init) <= 1e-6 * abs(e_init)
    # relative kinetic energy at the merger: fallen from d to a separation just inside s
    ke_contact = m * 2 * m * (1.0 / s - 1.0 / d)
    assert (1 - 1e-6) * ke_contact <= eps[0] <= 1.5 * ke_contact
    assert abs((eps[4] - eps[5]) - (eps[1] + eps[3])) <= 1e-12 * abs(eps[0])
    # hard energy: start = end + dissipated
    assert abs(r["e1"][0] + eps[5] - r["e0"][0]) <= 1e-5 * abs(r["e0"][0])


def compacted(n_clusters, seed, n_max, scale, eta):
    p = oracle.Params(eta=eta, eta0=0.1 * eta)
    d = diskgen.workload("disk64k_masslaw")
    ro, _, _ = oracle.cutoffs(d.pos, d.vel, d.mass, p)
    cl = diskgen.hermite_clusters(d, n_clusters=n_clusters, seed=seed, n_max=n_max, r_out=ro, compact=scale)
    return p, cl


def test_bookkeeping_on_compacted_clusters():
    """Many mergers (radius enhancement f = 200 on clusters compacted to
    0.7 r_out): per cluster, E_hard(start) - E_hard(end) - sum eps5 is the
    integration error alone (it falls with eta while the released energy
    stays), and the W / 1 - W / 1 identity holds."""
    gaps = {}
    for eta in (0.02, 0.001):
        p, cl = compacted(200, 4, 12, 0.7, eta)
        mem = np.arange(cl["pos"].shape[1], dtype=np.int32)
        r = oracle.hermite_collide(cl["pos"], cl["vel"], cl["mass"], cl["r_out"], cl["cl_ptr"], mem, p, 200.0, RHO)
        assert r["status"] == 0
        hit = r["ncoll"] > 0
        assert hit.sum() >= 100
        eps = r["eps"]
        scale = np.abs(r["e0"])
        gap = np.abs(r["e1"] + eps[:, 5] - r["e0"]) / scale
        released = np.abs(eps[:, 5]) / scale
        gaps[eta] = np.median(gap[hit])
        print(f"eta {eta}: clusters with mergers {hit.sum()}, mergers {r['ncoll'].sum()}, relative gap median "
              f"{gaps[eta]:.2e} max {gap[hit].max():.2e}, released / |E| median {np.median(released[hit]):.2e}")
        ident = np.abs((eps[:, 4] - eps[:, 5]) - (eps[:, 1] + eps[:, 3]))
        assert np.all(ident <= 1e-12 * (np.abs(eps[:, 4]) + np.abs(eps[:, 5]) + 1e-300))
        # merged_into names the lowest index of each composite, inside the cluster
        mi = r["merged_into"]
        assert np.all(mi <= mem) and np.all(mi[mi] == mi)
        for c in range(len(cl["cl_ptr"]) - 1):
            a, b = cl["cl_ptr"][c], cl["cl_ptr"][c + 1]
            assert np.all((mi[a:b] >= a) & (mi[a:b] < b))
            for s in np.unique(mi[a:b]):  # every composite's parts share one state
                parts = np.flatnonzero(mi == s)
                assert np.all(r["pos"][:, parts] == r["pos"][:, [s]]) and np.all(r["vel"][:, parts] == r["vel"][:, [s]])
        if eta == 0.001:
            assert gaps[eta] <= 1e-9 and np.median(released[hit]) >= 100 * gaps[eta]
    assert gaps[0.02] >= 10 * gaps[0.001]


def test_composite_moves_as_one_body():
    """Two touching bodies of equal cut-off merge at the first block step;
    from then on the composite and a third body follow the orbits of the
    two-body system with the merged body (plain Hermite from the merged
    state at t = 0); the only difference is the motion during that first
    step."""
    m1, m2, m3 = 1e-9, 2e-9, 1.5e-9
    R = radius(m1) + radius(m2)
    p = oracle.Params(eta=1e-3, eta0=1e-4, dt_soft=1.0 / 64)
    pos = np.array([[1.0, 1.0 + 0.5 * R, 1.0 + 3e-4], [0.0, 0.0, 1e-4], [0.0, 0.0, 0.0]])
    vel = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0 - 2e-4], [0.0, 0.0, 1e-5]])
    mass = np.array([m1, m2, m3])
    ro = np.full(3, 1e-3)
    dh = np.full(3, 1e-9)  # first block step tiny: the two parts barely move apart from the merged orbit
    r = oracle.hermite_collide(pos, vel, mass, ro, *one_cluster(3), p, 1.0, RHO, dt_hard=dh.copy())
    assert r["ncoll"][0] == 1 and np.array_equal(r["merged_into"], [0, 0, 2])
    M = m1 + m2
    xs = np.stack([(m1 * pos[:, 0] + m2 * pos[:, 1]) / M, pos[:, 2]], axis=1)
    vs = np.stack([(m1 * vel[:, 0] + m2 * vel[:, 1]) / M, vel[:, 2]], axis=1)
    x2, v2, _, _, _, st = oracle.hermite_clusters(xs, vs, np.array([M, m3]), ro[:2], *one_cluster(2), p)
    assert st == 0
    dx = np.abs(r["pos"][:, [0, 2]] - x2).max()
    dv = np.abs(r["vel"][:, [0, 2]] - v2).max()
    print("composite vs merged body: |dx|", dx, "|dv|", dv)
    assert dx < 1e-9 and dv < 1e-7
