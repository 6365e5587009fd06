"""Pins of the oracle P3T step (Section 2.2 steps (2)-(8), eq. (HamiltonSol))
and of the oracle leapfrog's forward pass, against results fixed by the
mathematics rather than by the oracle itself:

  * a lone planetesimal feels no soft force, so a step is its two-body
    orbit: a circular orbit turns by n dt (closed form);
  * the kick-hard-kick composition is symmetric, hence time-reversible:
    stepping forward, reversing the velocities and stepping again returns
    to the start (a kick with a stale force or a kick out of place breaks
    this);
  * the splitting is second order: with every pair beyond its cut-off
    (K = 1) the step is a kick-drift-kick map whose error against an
    accurate integration of the Newtonian equations (scipy DOP853) falls
    fourfold when dt halves (a wrong kick factor gives no convergence);
  * a pair closer than gamma r_out has K = 0: its whole force is in the
    hard part, and the step equals an accurate integration to the Hermite
    error; a pair inside the changeover converges at second order too;
  * the total energy (eq. (soft) + eq. (hard) = the Newtonian energy) of a
    pair inside the changeover is conserved up to a second-order splitting
    error;
  * the oracle leapfrog of the differentiable kick converges at second
    order on a circular orbit (closed form).
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import diskgen
from oracle import leapfrog as olf
from oracle import step as ostep


def newton_reference(pos, vel, mass, t_end, G=1.0, M=1.0):
    """Heliocentric planets about a fixed star with Newtonian mutual
    gravity (no changeover), integrated by scipy's DOP853 at rtol 1e-13."""
    n = mass.shape[0]

    def rhs(_t, y):
        x = y[:3 * n].reshape(3, n)
        v = y[3 * n:].reshape(3, n)
        r2 = (x * x).sum(0)
        a = -G * M * x / (r2 * np.sqrt(r2))
        for i in range(n):
            d = x - x[:, i:i + 1]
            rr = np.sqrt((d * d).sum(0))
            rr[i] = np.inf
            a[:, i] += G * (mass * d / rr**3).sum(1)
        return np.r_[v.ravel(), a.ravel()]

    y0 = np.r_[pos.ravel(), vel.ravel()]
    sol = solve_ivp(rhs, (0.0, t_end), y0, method="DOP853", rtol=1e-13, atol=1e-16)
    y = sol.y[:, -1]
    return y[:3 * n].reshape(3, n), y[3 * n:].reshape(3, n)


def circular(r, phi, z=0.0):
    vk = math.sqrt(1.0 / r)
    return (np.array([r * math.cos(phi), r * math.sin(phi), z]),
            np.array([-vk * math.sin(phi), vk * math.cos(phi), 0.0]))


def planets(specs):
    """(pos, vel) of planets on circular orbits given (r, phi) each."""
    xs, vs = zip(*(circular(r, ph) for r, ph in specs))
    return np.ascontiguousarray(np.stack(xs, 1)), np.ascontiguousarray(np.stack(vs, 1))


def run_to(pos, vel, mass, ro, rs, p, n_steps, isolated):
    s = ostep.init(pos, vel, mass, ro, rs, p)
    for _ in range(n_steps):
        s = ostep.step(s, mass, ro, rs, p, isolated)
        assert s.hermite_status == 0
    return s


@pytest.mark.parametrize("isolated", [1, 0])
def test_lone_particle_follows_its_circular_orbit(orc, isolated):
    p = orc.Params()
    x0, v0 = circular(1.3, 0.4)
    pos, vel = x0[:, None].copy(), v0[:, None].copy()
    m, ro, rs = np.array([1e-9]), np.array([1e-3]), np.array([2e-3])
    k = 5
    s = run_to(pos, vel, m, ro, rs, p, k, isolated)
    ang = 0.4 + k * p.dt_soft * math.sqrt(1.0 / 1.3**3)
    xe, ve = circular(1.3, ang)
    tol = 1e-13 if isolated else 1e-7  # Kepler drift is exact; Hermite (eta = 0.01) has its own error
    assert np.abs(s.pos[:, 0] - xe).max() < tol * 1.3
    assert np.abs(s.vel[:, 0] - ve).max() < tol
    assert np.all(s.acc == 0.0) and s.col.size == 0


def test_step_is_time_reversible(orc):
    """Forward k steps, reverse the velocities, k steps, reverse again: back
    to the start to rounding (Kepler drifts and symmetric kicks)."""
    p = orc.Params()
    pos, vel = planets([(1.0, 0.0), (1.08, 0.05), (0.93, -0.07)])
    m = np.array([3e-6, 1e-6, 2e-6])
    ro, rs = np.full(3, 1e-3), np.full(3, 2e-3)
    s = run_to(pos, vel, m, ro, rs, p, 4, isolated=1)
    assert s.col.size == 0 and np.abs(s.acc).max() > 1e-5  # no neighbours, real soft forces
    back = run_to(s.pos, -s.vel, m, ro, rs, p, 4, isolated=1)
    assert np.abs(back.pos - pos).max() < 1e-13
    assert np.abs(-back.vel - vel).max() < 1e-13
    # the forward map itself moved the planets by much more than that
    assert np.abs(s.pos - pos).max() > 0.1


def test_splitting_converges_at_second_order(orc):
    """Pairs beyond their cut-offs: K = 1, so the soft part is the whole
    mutual force and the hard part the Kepler drift.  The error against an
    accurate integration falls by 4 when dt halves."""
    pos, vel = planets([(1.0, 0.0), (1.06, 0.08), (0.95, -0.1)])
    m = np.array([2e-5, 1e-5, 3e-5])
    ro, rs = np.full(3, 1e-3), np.full(3, 2e-3)
    t_end = 16 * 2 * math.pi / 64
    xr, vr = newton_reference(pos, vel, m, t_end)
    errs = []
    for k in (16, 32, 64):
        p = orc.Params(dt_soft=t_end / k)
        s = run_to(pos, vel, m, ro, rs, p, k, isolated=1)
        errs.append(np.abs(s.pos - xr).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    print("splitting errors", errs, "ratios", r1, r2)
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4
    assert errs[0] < 1e-4  # small against the mutual perturbation (~1e-2 au over the run)


def pair_state(sep, rel_v=0.0):
    """Two planets near 1 au, sep apart radially, with circular velocities
    plus a small relative tangential velocity."""
    pos, vel = planets([(1.0, 0.0), (1.0 + sep, 0.0)])
    vel[1, 1] += rel_v
    return pos, vel


def test_pair_inside_inner_radius_is_all_hard(orc):
    """y < gamma: K = 0, the soft force between the pair vanishes and the
    step is the Hermite integration of the star plus the full pair force."""
    m = np.array([1e-7, 1e-7])
    sep = 2e-3
    ro = np.full(2, 0.1)  # gamma r_out = 1e-2 > sep over the whole run
    rs = np.full(2, 0.2)
    pos, vel = pair_state(sep, rel_v=-2e-4)
    p = orc.Params(eta=1e-4, eta0=1e-5)
    k = 4
    s = run_to(pos, vel, m, ro, rs, p, k, isolated=0)
    assert np.all(s.acc == 0.0)  # the soft part of a pair at y < gamma
    assert s.n_clusters == 1
    xr, vr = newton_reference(pos, vel, m, k * p.dt_soft)
    rel = s.pos - xr
    d = s.pos[:, 1] - s.pos[:, 0]
    dr = xr[:, 1] - xr[:, 0]
    print("inner pair: abs err", np.abs(rel).max(), "separation err", np.abs(d - dr).max() / np.linalg.norm(dr))
    assert np.abs(rel).max() < 1e-10
    assert np.abs(d - dr).max() < 1e-6 * np.linalg.norm(dr)


def test_pair_in_changeover_converges_and_conserves_energy(orc):
    """A pair inside the changeover region (gamma r_out < r < r_out): part
    of its force is kicked, the rest integrated; the step converges at
    second order to the Newtonian motion and conserves the total energy."""
    m = np.array([3e-7, 2e-7])
    sep = 1.2e-2
    ro, rs = np.full(2, 2.4e-2), np.full(2, 4e-2)  # y = 0.5 at the start
    pos, vel = pair_state(sep, rel_v=1e-4)
    t_end = 8 * 2 * math.pi / 64
    xr, _ = newton_reference(pos, vel, m, t_end)
    errs, e_err = [], []
    for k in (8, 16, 32):
        p = orc.Params(dt_soft=t_end / k, eta=1e-4, eta0=1e-5)
        s = ostep.init(pos, vel, m, ro, rs, p)
        E0 = ostep.total_energy(pos, vel, m, p)
        worst = 0.0
        for _ in range(k):
            s = ostep.step(s, m, ro, rs, p, 0)
            assert s.n_clusters == 1 and s.hermite_status == 0
            worst = max(worst, abs(ostep.total_energy(s.pos, s.vel, m, p) - E0) / abs(E0))
        d = np.linalg.norm(s.pos[:, 1] - s.pos[:, 0])
        assert 0.1 * ro[0] < d < ro[0]  # still in the changeover
        errs.append(np.abs(s.pos - xr).max())
        e_err.append(worst)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    print("changeover pair errors", errs, "ratios", r1, r2, "energy", e_err)
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7
    # the splitting's energy error is second order too, and small against
    # the pair's own interaction energy
    assert 3.3 < e_err[0] / e_err[1] < 4.7 and 3.3 < e_err[1] / e_err[2] < 4.7
    E_abs = abs(ostep.total_energy(pos, vel, m, p))
    assert max(e_err) * E_abs < 1e-2 * m[0] * m[1] / sep


def test_oracle_step_on_a_disk_keeps_energy(orc):
    """A small equal-mass disk with its radii from eq. (routi2) over a few
    steps: the total energy changes by a small fraction of the mutual
    interaction energy."""
    d = diskgen.make_disk(256, 0.995, 1.005, seed=12, m_equal=1e-8)
    p = orc.Params(r_cut0=3.0)
    ro, rs, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
    s = ostep.init(d.pos, d.vel, d.mass, ro, rs, p)
    E0 = ostep.total_energy(d.pos, d.vel, d.mass, p)
    n_pairs = [s.col.size]
    for _ in range(4):
        s = ostep.step(s, d.mass, ro, rs, p, 1)
        assert s.hermite_status == 0
        n_pairs.append(s.col.size)
    E1 = ostep.total_energy(s.pos, s.vel, d.mass, p)
    # the mutual (pair) part of the energy: the total with the star's mass
    # and the kinetic terms taken out
    kin = 0.5 * float((d.mass * (d.vel * d.vel).sum(0)).sum())
    U = ostep.total_energy(d.pos, np.zeros_like(d.vel), d.mass, orc.Params(m_star=0.0))
    print("disk256: pairs per step", n_pairs, "energy error", abs(E1 - E0) / abs(E0), "of U", abs(E1 - E0) / abs(U),
          "kinetic", kin)
    assert max(n_pairs) > 0
    assert abs(E1 - E0) < 1e-2 * abs(U)


def test_leapfrog_forward_converges_at_second_order(orc):
    """The oracle leapfrog (soft kick, star kick, linear drift) on a lone
    circular orbit against its closed form: errors fall fourfold per
    halving of the step."""
    x0, v0 = circular(1.0, 0.3)
    t_end = 2.0
    xe, _ = circular(1.0, 0.3 + t_end)
    p = orc.Params()
    errs = []
    for k in (32, 64, 128):
        h = t_end / k
        xf, _, _ = olf.leapfrog(x0[:, None].copy(), v0[:, None].copy(), np.array([1e-9]), np.array([1e-3]), p, h, k)
        errs.append(np.abs(xf[:, 0] - xe).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2


def test_sparse_bin_takes_the_global_rms(orc):
    """A dense ring on circular orbits (no random velocity) and three lone
    particles far outside it with a known vertical random velocity: the
    lone particles' bin has fewer than vran_min_count members, so they get
    the rms over all particles, sqrt(3 u^2 / n); the ring keeps zero."""
    rng = np.random.default_rng(5)
    n_ring, u = 1000, 4e-3
    r = np.r_[rng.uniform(0.9, 0.95, n_ring), [2.0, 2.01, 2.02]]
    phi = rng.uniform(0, 2 * math.pi, n_ring + 3)
    pos = np.stack([r * np.cos(phi), r * np.sin(phi), np.zeros(n_ring + 3)])
    vk = np.sqrt(1.0 / r)
    vz = np.r_[np.zeros(n_ring), np.full(3, u)]
    vel = np.stack([-vk * np.sin(phi), vk * np.cos(phi), vz])
    m = np.full(n_ring + 3, 1e-12)
    p = orc.Params(vran_bins=8, vran_min_count=8)
    _, _, vr = orc.cutoffs(pos, vel, m, p)
    assert np.all(vr[:n_ring] < 1e-15)
    assert np.allclose(vr[n_ring:], math.sqrt(3 * u * u / (n_ring + 3)), rtol=1e-12)
    # with a threshold of 3 the lone bin is its own rms
    _, _, vr3 = orc.cutoffs(pos, vel, m, orc.Params(vran_bins=8, vran_min_count=3))
    assert np.allclose(vr3[n_ring:], u, rtol=1e-12)


def test_shared_cutoff_takes_the_largest_radii(orc):
    """Shared mode (eq. (rout1); shared search radius of Section 2.3): two
    rings with known random velocities, the outer ring's velocity term the
    largest: every particle gets r_out = Rcut1 u_out dt and r_search =
    Rsearch0 r_out + Rsearch1 u_out dt, while v_ran stays per bin."""
    n = 1000
    rng = np.random.default_rng(2)
    r = np.r_[rng.uniform(0.9, 0.95, n), rng.uniform(2.0, 2.1, n)]
    phi = rng.uniform(0, 2 * math.pi, 2 * n)
    pos = np.stack([r * np.cos(phi), r * np.sin(phi), np.zeros(2 * n)])
    vk = np.sqrt(1.0 / r)
    u_in, u_out = 1e-3, 4e-3
    vel = np.stack([-vk * np.sin(phi), vk * np.cos(phi), np.r_[np.full(n, u_in), np.full(n, u_out)]])
    m = np.full(2 * n, 1e-12)
    p = orc.Params(vran_bins=8, cutoff_mode=1)
    ro, rs, vr = orc.cutoffs(pos, vel, m, p)
    ro_exp = p.r_cut1 * u_out * p.dt_soft
    assert np.allclose(ro, ro_exp, rtol=1e-14)
    assert np.allclose(rs, p.r_search0 * ro_exp + p.r_search1 * u_out * p.dt_soft, rtol=1e-14)
    assert np.allclose(vr[:n], u_in, rtol=1e-12) and np.allclose(vr[n:], u_out, rtol=1e-12)
    # individual mode on the same input: the inner ring keeps its own radii
    ro_i, _, _ = orc.cutoffs(pos, vel, m, orc.Params(vran_bins=8))
    assert np.allclose(ro_i[:n], p.r_cut1 * u_in * p.dt_soft, rtol=1e-14)
    assert ro_i.max() == ro.max()
