"""Pins of the oracle leapfrog adjoint (used as the reference gradient of the
differentiable soft kick): central finite differences of the oracle's own
leapfrog loss, and translation of the initial state."""
import numpy as np
import pytest

import diskgen
from oracle import leapfrog as olf


@pytest.fixture(scope="module")
def system(orc):
    d = diskgen.make_disk(40, 0.999, 1.001, seed=21, m_min=1e-10, m_max=1e-8)
    rng = np.random.default_rng(8)
    ro = rng.uniform(5e-4, 3e-3, d.n)
    return d, ro, orc.Params()


def dloss(d, ro, p, plus, minus, h, steps):
    """L(plus) - L(minus) for L = sum |x_final|^2, formed per element as
    (a - b)(a + b) so that unchanged coordinates cancel exactly."""
    a = olf.leapfrog(*plus, ro, p, h, steps)[0]
    b = olf.leapfrog(*minus, ro, p, h, steps)[0]
    return float(((a - b) * (a + b)).sum())


def test_leapfrog_adjoint_matches_finite_differences(orc, system):
    d, ro, p = system
    h, steps = p.dt_soft, 3
    xf, vf, tape = olf.leapfrog(d.pos, d.vel, d.mass, ro, p, h, steps)
    lx, lv, lm = olf.leapfrog_adjoint(d.mass, ro, p, h, tape, 2.0 * xf, np.zeros_like(vf))
    for k in (0, 17, 39):
        for c in range(3):
            e = 1e-7
            xp, xm = d.pos.copy(), d.pos.copy()
            xp[c, k] += e
            xm[c, k] -= e
            fd = dloss(d, ro, p, (xp, d.vel, d.mass), (xm, d.vel, d.mass), h, steps) / (2 * e)
            assert abs(fd - lx[c, k]) < 1e-6 * abs(lx).max(), (k, c, fd, lx[c, k])
            vp, vm = d.vel.copy(), d.vel.copy()
            vp[c, k] += e
            vm[c, k] -= e
            fd = dloss(d, ro, p, (d.pos, vp, d.mass), (d.pos, vm, d.mass), h, steps) / (2 * e)
            assert abs(fd - lv[c, k]) < 1e-6 * abs(lv).max(), (k, c, fd, lv[c, k])
        dm = 1e-3 * d.mass[k]  # smaller steps drown in the rounding of x (|dx| ~ 1e-14)
        mp, mm = d.mass.copy(), d.mass.copy()
        mp[k] += dm
        mm[k] -= dm
        fd = dloss(d, ro, p, (d.pos, d.vel, mp), (d.pos, d.vel, mm), h, steps) / (2 * dm)
        assert abs(fd - lm[k]) < 1e-5 * abs(lm).max(), (k, fd, lm[k])


def test_mass_gradient_vanishes_without_interactions(orc, system):
    """A single particle feels no soft force, so its mass has no gradient,
    while the star-only orbit still has a finite position gradient."""
    d, ro, p = system
    x, v, m = d.pos[:, :1].copy(), d.vel[:, :1].copy(), d.mass[:1].copy()
    xf, vf, tape = olf.leapfrog(x, v, m, ro[:1], p, p.dt_soft, 2)
    lx, lv, lm = olf.leapfrog_adjoint(m, ro[:1], p, p.dt_soft, tape, 2.0 * xf, np.zeros_like(vf))
    assert lm[0] == 0.0
    assert np.all(np.isfinite(lx)) and np.all(np.isfinite(lv))


def test_forward_two_body_converges_at_second_order(orc):
    """Forward pin of the kick-drift-kick steps, apart from the adjoint: two
    bodies beyond their cut-offs (K = 1, the whole Newtonian pair force) and
    no star move as a Kepler pair about their centre of mass.  The relative
    orbit after a fixed time, against the oracle's Kepler drift with
    mu = G (m1 + m2), converges at second order in the step; a kick of the
    wrong weight or a drift with a stale velocity would not."""
    from oracle.kepler import kepler_drift

    p = orc.Params()
    m = np.array([3e-6, 1e-6])
    M = m.sum()
    mu = p.G * M
    a = 0.01
    rel_x = np.array([a, 0.0, 0.0])
    rel_v = np.array([0.0, 1.2 * np.sqrt(mu / a), 0.1 * np.sqrt(mu / a)])  # bound, e ~ 0.45, inclined
    com_x, com_v = np.array([1.0, 0.5, 0.0]), np.array([0.01, -0.02, 0.0])
    x = np.stack([com_x - m[1] / M * rel_x, com_x + m[0] / M * rel_x], axis=1)
    v = np.stack([com_v - m[1] / M * rel_v, com_v + m[0] / M * rel_v], axis=1)
    ro = np.array([1e-5, 1e-5])  # far inside the separation: y >> 1, K = 1
    energy = 0.5 * (rel_v @ rel_v) - mu / a
    period = 2.0 * np.pi * np.sqrt((-mu / (2.0 * energy)) ** 3 / mu)
    t_end = 0.37 * period
    xr, vr, bound, _ = kepler_drift(rel_x[:, None], rel_v[:, None], mu, t_end)
    assert bound.all()

    def rel_error(n):
        xf, vf, _ = olf.leapfrog(x, v, m, ro, p, t_end / n, n, GM=0.0)
        got = xf[:, 1] - xf[:, 0]
        com = (m[0] * xf[:, 0] + m[1] * xf[:, 1]) / M
        assert np.abs(com - (com_x + t_end * com_v)).max() < 1e-13  # momentum is conserved exactly
        return np.abs(got - xr[:, 0]).max() / a

    e = [rel_error(n) for n in (400, 800, 1600)]
    for e1, e2 in zip(e, e[1:]):
        assert 3.6 < e1 / e2 < 4.4, e
    assert e[-1] < 1e-4


def test_forward_star_orbit_converges_at_second_order(orc):
    """The star's kicks and the drift alone: one particle with no partner
    on an eccentric orbit about the star, against the Kepler drift with
    mu = GM; the error falls fourfold when the step halves."""
    from oracle.kepler import kepler_drift

    p = orc.Params()
    x = np.array([[1.0], [0.1], [0.02]])
    v = np.array([[0.05], [1.1], [0.03]])
    t_end = 1.3
    xr, vr, bound, _ = kepler_drift(x, v, 1.0, t_end)
    assert bound.all()
    e = []
    for n in (200, 400, 800):
        xf, vf, _ = olf.leapfrog(x, v, np.array([1e-9]), np.array([1e-3]), p, t_end / n, n, GM=1.0)
        e.append(np.abs(xf - xr).max())
    for e1, e2 in zip(e, e[1:]):
        assert 3.6 < e1 / e2 < 4.4, e
    assert e[-1] < 1e-4
