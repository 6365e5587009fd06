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
