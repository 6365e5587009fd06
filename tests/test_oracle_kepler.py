"""Pins of the oracle Kepler drift (oracle/kepler.py) against closed forms and
an independent integrator.

  * circular orbit: a rotation by n dt, written out;
  * eccentric orbit from pericentre: apocentre a(1 + e) after half a period,
    back to the start after a full period;
  * energy and angular momentum conserved for random bound states;
  * two drifts compose into one;
  * a single particle against the oracle's Hermite integrator (star only),
    to the Hermite's own accuracy;
  * the disk generator's elements advanced in mean anomaly by n dt (its own
    Kepler solver on the anomaly itself, not on its difference);
  * an unbound state, and one at the star's position, are left alone and
    reported.
"""
import math

import numpy as np
import pytest

import diskgen

from oracle.kepler import kepler_drift

MU = 1.0


def test_circular_orbit_is_a_rotation():
    R = 1.3
    x0 = np.array([[R], [0.0], [0.0]])
    v0 = np.array([[0.0], [math.sqrt(MU / R)], [0.0]])
    n = math.sqrt(MU / R ** 3)
    for dt in (0.01, 0.7, 5.0, 40.0):
        x, v, ok, _ = kepler_drift(x0, v0, MU, dt)
        assert ok.all()
        ref = R * np.array([math.cos(n * dt), math.sin(n * dt), 0.0])
        vref = math.sqrt(MU / R) * np.array([-math.sin(n * dt), math.cos(n * dt), 0.0])
        assert np.abs(x[:, 0] - ref).max() < 1e-13 * R
        assert np.abs(v[:, 0] - vref).max() < 1e-13


@pytest.mark.parametrize("e", [0.1, 0.5, 0.9])
def test_pericentre_to_apocentre_and_back(e):
    a = 2.0
    rp = a * (1 - e)
    vp = math.sqrt(MU * (1 + e) / (a * (1 - e)))
    # inclined orbit plane: pericentre along x, velocity in the y-z plane
    inc = 0.3
    x0 = np.array([[rp], [0.0], [0.0]])
    v0 = np.array([[0.0], [vp * math.cos(inc)], [vp * math.sin(inc)]])
    P = 2 * math.pi * math.sqrt(a ** 3 / MU)
    x, v, ok, _ = kepler_drift(x0, v0, MU, 0.5 * P)
    assert ok.all()
    assert abs(x[0, 0] + a * (1 + e)) < 1e-12 * a and abs(x[1, 0]) < 1e-11 * a and abs(x[2, 0]) < 1e-11 * a
    x, v, _, _ = kepler_drift(x0, v0, MU, P)
    assert np.abs(x - x0).max() < 1e-11 * a and np.abs(v - v0).max() < 1e-11 * vp


def random_bound(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(3, n))
    x *= rng.uniform(0.5, 5.0, n) / np.sqrt((x * x).sum(0))
    r = np.sqrt((x * x).sum(0))
    v = rng.normal(size=(3, n))
    v *= rng.uniform(0.2, 1.35, n) * np.sqrt(MU / r) / np.sqrt((v * v).sum(0))  # |v| < sqrt(2 mu / r): bound
    return x, v


def test_energy_and_angular_momentum_conserved():
    x0, v0 = random_bound(500, 3)
    x, v, ok, it = kepler_drift(x0, v0, MU, 0.37)
    assert ok.all() and it.max() < 50

    def energy(x, v):
        return 0.5 * (v * v).sum(0) - MU / np.sqrt((x * x).sum(0))

    e0, e1 = energy(x0, v0), energy(x, v)
    assert np.abs((e1 - e0) / e0).max() < 1e-12
    L0, L1 = np.cross(x0.T, v0.T), np.cross(x.T, v.T)
    assert np.abs(L1 - L0).max() < 1e-12 * np.abs(L0).max()


def test_drifts_compose():
    x0, v0 = random_bound(200, 4)
    x1, v1, _, _ = kepler_drift(x0, v0, MU, 0.2)
    x2, v2, _, _ = kepler_drift(x1, v1, MU, 0.3)
    x3, v3, _, _ = kepler_drift(x0, v0, MU, 0.5)
    assert np.abs(x2 - x3).max() < 1e-12 * np.abs(x3).max()
    assert np.abs(v2 - v3).max() < 1e-12 * np.abs(v3).max()


def test_single_particle_matches_the_hermite_oracle(orc):
    """One isolated particle: the oracle's fourth-order Hermite (star only,
    block steps at eta = 0.02) against the exact drift."""
    p = orc.Params()
    rng = np.random.default_rng(5)
    n = 16
    a = rng.uniform(0.6, 1.4, n)
    e = rng.uniform(0.0, 0.2, n)
    M = rng.uniform(0, 2 * math.pi, n)
    E = M.copy()
    for _ in range(50):
        E = E - (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    GM = p.G * p.m_star
    r = a * (1 - e * np.cos(E))
    x = np.stack([a * (np.cos(E) - e), a * np.sqrt(1 - e * e) * np.sin(E), np.zeros(n)])
    v = np.stack([-np.sqrt(GM * a) / r * np.sin(E), np.sqrt(GM * a * (1 - e * e)) / r * np.cos(E), np.zeros(n)])
    mass = np.full(n, 1e-12)
    ro = np.full(n, 1e-6)
    cl_ptr = np.arange(n + 1, dtype=np.int32)
    members = np.arange(n, dtype=np.int32)
    xh, vh, *_ = orc.hermite_clusters(x, v, mass, ro, cl_ptr, members, p)
    xk, vk, ok, _ = kepler_drift(x, v, GM, p.dt_soft)
    assert ok.all()
    err = np.abs(xh - xk).max() / np.abs(xk).max()
    print("Hermite vs exact drift over one soft step:", err)
    assert err < 1e-8


def test_unbound_state_is_left_alone():
    x0 = np.array([[1.0], [0.0], [0.0]])
    v0 = np.array([[0.0], [1.6], [0.0]])  # above escape speed sqrt(2)
    x, v, ok, _ = kepler_drift(x0, v0, MU, 0.5)
    assert not ok[0] and np.array_equal(x, x0) and np.array_equal(v, v0)


def test_state_at_the_advanced_mean_anomaly():
    """elements_to_state at M + n dt against a drift from the state at M:
    two different routes through Kepler's equation."""
    d = diskgen.workload("disk64k_masslaw", n=4096)
    rng = np.random.default_rng(9)
    inc = d.inc
    Om, om, M = (rng.random(d.n) * 2 * math.pi for _ in range(3))
    e = np.minimum(d.e * 30.0, 0.8)  # a wider spread of eccentricities than the disk's
    x0, v0 = diskgen.elements_to_state(d.a, e, inc, Om, om, M)
    for dt in (1.0 / 64, 0.9, 7.0):
        nm = np.sqrt(1.0 / d.a ** 3)
        x1, v1 = diskgen.elements_to_state(d.a, e, inc, Om, om, M + nm * dt)
        x, v, ok, _ = kepler_drift(x0, v0, 1.0, dt)
        assert ok.all()
        assert np.abs(x - x1).max() < 1e-11 * np.abs(x1).max(), dt
        assert np.abs(v - v1).max() < 1e-11 * np.abs(v1).max(), dt


def test_state_at_the_star_is_left_alone():
    x0 = np.zeros((3, 1))
    v0 = np.array([[0.1], [0.0], [0.0]])
    x, v, ok, _ = kepler_drift(x0, v0, MU, 0.5)
    assert not ok[0] and np.array_equal(x, x0) and np.array_equal(v, v0)
