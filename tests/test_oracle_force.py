"""Pins for the oracle's soft acceleration (eq. (softforce) with the pair
cut-off of eq. (rout2)) and hard acceleration / jerk (eq. (hardforce)).

Pinned against:
  * the force-from-potential relation: a_soft,i = -(1/m_i) dH_soft/dx_i with
    H_soft of eq. (soft), differentiated numerically (ties the force's K to
    the Hamiltonian's W, catches sign / index / mass-subscript mistakes);
  * soft + hard pair parts = Newtonian gravity, against a numpy Newtonian sum
    (eq. (softforce) + eq. (hardforce));
  * Newton's third law (pairwise antisymmetry because r_out,ij is symmetric);
  * the limits K = 1 (all pairs beyond r_out: plain Newton) and K = 0 (all
    pairs inside r_in: no soft force);
  * a two-body configuration at a known y against the closed form of K;
  * the jerk against a finite difference of the acceleration along the
    motion, including the dK/dt term.
"""
import math

import numpy as np
import pytest

import diskgen


def _newton_numpy(pos, m, G=1.0):
    d = pos[:, None, :] - pos[:, :, None]  # d[:, i, j] = x_j - x_i
    r2 = (d**2).sum(0)
    np.fill_diagonal(r2, np.inf)
    return (G * m[None, None, :] * d / r2[None] ** 1.5).sum(-1)


@pytest.fixture(scope="module")
def cluster():
    """A compact blob of 40 planetesimals at 1 au with r_out comparable to
    the separations, so pairs fall in all three changeover regimes."""
    rng = np.random.default_rng(7)
    n = 40
    pos = np.array([1.0, 0.0, 0.0])[:, None] + rng.normal(0, 2e-3, (3, n)) * np.array([[1], [1], [0.2]])
    m = rng.uniform(0.5e-9, 2e-9, n)
    r_out = rng.uniform(1e-3, 3e-3, n)
    return np.ascontiguousarray(pos), m, r_out


def test_newton_numpy_matches_oracle(orc, cluster):
    pos, m, _ = cluster
    assert np.allclose(orc.newton_acc(pos, m), _newton_numpy(pos, m), rtol=1e-12, atol=0)


def test_soft_is_gradient_of_soft_hamiltonian(orc, params, cluster):
    pos, m, ro = cluster
    a = orc.soft_acc(pos, m, ro, params)
    # regime check: some pairs in each of K = 0, 0 < K < 1, K = 1
    d = np.sqrt(((pos[:, :, None] - pos[:, None, :]) ** 2).sum(0))
    y = d / np.maximum(ro[:, None], ro[None, :])
    iu = np.triu_indices(len(m), 1)
    assert (y[iu] < params.gamma).any() and ((y[iu] > params.gamma) & (y[iu] < 1)).any() and (y[iu] > 1).any()
    h = 1e-9
    for i in [0, 3, 17, 39]:
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[c, i] += h
            pm[c, i] -= h
            g = (orc.soft_energy(pp, m, ro, params) - orc.soft_energy(pm, m, ro, params)) / (2 * h)
            assert abs(-g / m[i] - a[c, i]) <= 2e-6 * np.abs(a[:, i]).max() + 1e-12


def test_soft_plus_hard_is_newton(orc, cluster):
    pos, m, ro = cluster
    p = orc.Params(m_star=0.0)  # no star: the hard part is the (1-K) pair sum alone
    vel = np.zeros_like(pos)
    a_soft = orc.soft_acc(pos, m, ro, p)
    a_hard, _ = orc.hard_acc_jerk(pos, vel, m, ro, p)
    a_newt = _newton_numpy(pos, m)
    assert np.max(np.abs(a_soft + a_hard - a_newt)) <= 1e-13 * np.max(np.abs(a_newt))


def test_momentum_antisymmetry(orc, params):
    d = diskgen.make_disk(512, 0.9, 1.1, seed=21, m_min=1e-10, m_max=1e-8)
    ro, rs, _ = orc.cutoffs(d.pos, d.vel, d.mass, params)
    ro = ro * 20.0  # widen so that many pairs are inside the changeover region
    a = orc.soft_acc(d.pos, d.mass, ro, params)
    tot = (d.mass[None] * a).sum(1)
    scale = (d.mass[None] * np.abs(a)).sum(1)
    assert np.all(np.abs(tot) <= 1e-13 * scale)


def test_newton_limit_and_zero_limit(orc, params, cluster):
    pos, m, _ = cluster
    tiny = np.full(len(m), 1e-9)
    assert np.allclose(orc.soft_acc(pos, m, tiny, params), _newton_numpy(pos, m), rtol=1e-13, atol=0)
    huge = np.full(len(m), 10.0)
    assert np.all(orc.soft_acc(pos, m, huge, params) == 0.0)


def test_two_body_closed_form(orc, params):
    g = params.gamma
    r, R = 2.0**-10, 2.0**-9  # exactly representable, y = 0.5
    pos = np.array([[1.0, 1.0 + r], [0.0, 0.0], [0.0, 0.0]])
    m = np.array([1e-9, 3e-9])
    ro = np.array([R, 0.5 * R])  # pair cut-off is the larger one
    a = orc.soft_acc(pos, m, ro, params)
    x = (0.5 - g) / (1 - g)
    K = 35 * x**4 - 84 * x**5 + 70 * x**6 - 20 * x**7
    assert math.isclose(a[0, 0], 3e-9 * K / r**2, rel_tol=1e-13)
    assert math.isclose(a[0, 1], -1e-9 * K / r**2, rel_tol=1e-13)
    assert a[1, 0] == 0.0 and a[2, 1] == 0.0


def test_jerk_is_time_derivative(orc, params, cluster):
    pos, m, ro = cluster
    rng = np.random.default_rng(3)
    vel = np.array([0.0, 1.0, 0.0])[:, None] + rng.normal(0, 1e-3, pos.shape)
    a, j = orc.hard_acc_jerk(pos, vel, m, ro, params)
    h = 1e-7
    ap, _ = orc.hard_acc_jerk(pos + h * vel, vel, m, ro, params)
    am, _ = orc.hard_acc_jerk(pos - h * vel, vel, m, ro, params)
    fd = (ap - am) / (2 * h)
    scale = np.abs(j).max(axis=0)
    assert np.all(np.abs(fd - j) <= 1e-5 * scale[None] + 1e-10)


def test_subset_rows_equal_full(orc, params, cluster):
    pos, m, ro = cluster
    full = orc.soft_acc(pos, m, ro, params)
    idx = np.array([5, 1, 30])
    assert np.array_equal(orc.soft_acc(pos, m, ro, params, idx=idx), full[:, idx])
