"""Pins for the oracle's cut-off radii (Hill radius, eq. (routi2), eq.
(rsearch)) and its soft-force vector-Jacobian product.

Cut-offs are pinned against the generator's own orbital elements (the
osculating semi-major axis from vis-viva equals the drawn a), circular orbits
(zero random velocity), constructed random velocities and the rotation
invariance about the star's axis.  The VJP is pinned against central finite
differences of the oracle's forward force and against translation
invariance (sum_k dL/dx_k = 0).
"""
import math

import numpy as np
import pytest

import diskgen


def test_hill_term_uses_semimajor_axis(orc):
    d = diskgen.make_disk(3000, 0.5, 1.5, seed=2)
    p = orc.Params(r_cut1=0.0, r_search1=0.0)
    ro, rs, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
    a_back = ro / (p.r_cut0 * np.cbrt(d.mass / 3.0))
    assert np.allclose(a_back, d.a, rtol=1e-10, atol=0)
    assert np.allclose(rs, p.r_search0 * ro, rtol=1e-15, atol=0)
    p1 = orc.Params(r_cut1=0.0, r_search1=0.0, hill_length=1)
    ro1, _, _ = orc.cutoffs(d.pos, d.vel, d.mass, p1)
    assert np.allclose(ro1 / (p.r_cut0 * np.cbrt(d.mass / 3.0)), np.sqrt((d.pos**2).sum(0)), rtol=1e-14)


def test_circular_orbits_have_no_random_velocity(orc):
    n = 500
    rng = np.random.default_rng(1)
    r = rng.uniform(0.8, 1.2, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    pos = np.stack([r * np.cos(phi), r * np.sin(phi), np.zeros(n)])
    vk = np.sqrt(1.0 / r)
    vel = np.stack([-vk * np.sin(phi), vk * np.cos(phi), np.zeros(n)])
    m = np.full(n, 1e-9)
    p = orc.Params()
    ro, rs, vr = orc.cutoffs(pos, vel, m, p)
    assert np.all(vr < 1e-15)
    assert np.allclose(ro, p.r_cut0 * np.cbrt(m / 3.0) * r, rtol=1e-12)


def test_random_velocity_by_radial_bin(orc):
    """Two rings with different, known random velocities: each particle's v_ran
    is its own ring's rms, and the velocity term sets r_out where it dominates."""
    n = 1000
    rng = np.random.default_rng(2)
    r = np.r_[rng.uniform(0.9, 0.95, n), rng.uniform(2.0, 2.1, n)]
    phi = rng.uniform(0, 2 * math.pi, 2 * n)
    pos = np.stack([r * np.cos(phi), r * np.sin(phi), np.zeros(2 * n)])
    vk = np.sqrt(1.0 / r)
    dv = np.r_[np.full(n, 1e-3), np.full(n, 4e-3)]
    vel = np.stack([-vk * np.sin(phi), vk * np.cos(phi), dv])  # random part purely vertical
    m = np.full(2 * n, 1e-12)
    p = orc.Params(vran_bins=8)
    ro, rs, vr = orc.cutoffs(pos, vel, m, p)
    assert np.allclose(vr[:n], 1e-3, rtol=1e-12) and np.allclose(vr[n:], 4e-3, rtol=1e-12)
    assert np.allclose(ro, p.r_cut1 * vr * p.dt_soft, rtol=1e-14)
    assert np.allclose(rs, p.r_search0 * ro + p.r_search1 * vr * p.dt_soft, rtol=1e-14)


def test_cutoffs_rotation_invariant(orc, params):
    d = diskgen.workload("disk2k_equal")
    ro, rs, vr = orc.cutoffs(d.pos, d.vel, d.mass, params)
    c, s = math.cos(0.7), math.sin(0.7)
    Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    ro2, rs2, vr2 = orc.cutoffs(Rz @ d.pos, Rz @ d.vel, d.mass, params)
    assert np.allclose(ro, ro2, rtol=1e-9) and np.allclose(rs, rs2, rtol=1e-9)


def test_config1_scales(orc, params):
    """At the equal-mass 0.9-1.1 au disk the Hill term dominates (rms e = 2h)."""
    d = diskgen.workload("disk2k_equal")
    ro, rs, vr = orc.cutoffs(d.pos, d.vel, d.mass, params)
    h = diskgen.reduced_hill(1e-9)
    assert 1.0e-3 < np.median(ro) < 2.0e-3
    assert np.all(ro >= params.r_cut0 * h * 0.85)
    assert 0.5 * 2 * h < np.median(vr) < 2 * 2 * h  # rms random velocity ~ rms e * v_K


@pytest.fixture(scope="module")
def small_system():
    d = diskgen.make_disk(48, 0.999, 1.001, seed=9, m_min=1e-10, m_max=1e-8)
    rng = np.random.default_rng(4)
    ro = rng.uniform(5e-4, 3e-3, d.n)
    lam = rng.normal(0, 1, (3, d.n))
    return d, ro, lam


def test_adjoint_matches_finite_differences(orc, params, small_system):
    d, ro, lam = small_system
    gp, gm = orc.soft_adjoint(d.pos, d.mass, ro, lam, params)

    def L(pos, m):
        return float((lam * orc.soft_acc(pos, m, ro, params)).sum())

    scale_x = np.abs(gp).max()
    for k in [0, 5, 23, 47]:
        for c in range(3):
            h = 1e-8
            pp, pm = d.pos.copy(), d.pos.copy()
            pp[c, k] += h
            pm[c, k] -= h
            fd = (L(pp, d.mass) - L(pm, d.mass)) / (2 * h)
            assert abs(fd - gp[c, k]) < 1e-5 * scale_x
        hm = 1e-6 * d.mass[k]
        mp_, mm_ = d.mass.copy(), d.mass.copy()
        mp_[k] += hm
        mm_[k] -= hm
        fd = (L(d.pos, mp_) - L(d.pos, mm_)) / (2 * hm)
        assert abs(fd - gm[k]) < 1e-7 * np.abs(gm).max()


def test_adjoint_translation_invariance(orc, params, small_system):
    d, ro, lam = small_system
    gp, _ = orc.soft_adjoint(d.pos, d.mass, ro, lam, params)
    assert np.all(np.abs(gp.sum(1)) < 1e-10 * np.abs(gp).sum(1))
