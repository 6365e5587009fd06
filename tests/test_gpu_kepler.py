"""GPU parity of p3t_kepler_drift (Section 2.2: particles without neighbours
move on their two-body orbits) against the oracle's drift.

  * bound orbits over a soft step and over several orbital periods: positions
    and velocities to 1e-12 of their scale (both sides converge Newton's
    method to 1e-15 in FP64; the rest is a few roundings of sin and cos),
    Newton iteration counts within one of the oracle's;
  * a list drifts only its own particles: the others stay bit for bit;
  * unbound states and a state at the star are left bit for bit and counted;
  * empty list, all-particle form without a list, a list entry out of range;
  * the 2^20-particle disk, every particle drifted, checked on a sample.
"""
import math

import numpy as np
import pytest
import torch

import diskgen
from oracle.kepler import kepler_drift

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def ctx(gpu, orc):
    p = orc.Params()
    c = gpu.Context(gpu.Params.defaults().replace(G=p.G, m_star=p.m_star, dt_soft=p.dt_soft))
    yield c
    c.close()


def states(n, seed):
    """Disk orbits; every third one given an eccentricity up to 0.9."""
    d = diskgen.workload("disk64k_masslaw", n=n)
    rng = np.random.default_rng(seed)
    e = d.e.copy()
    e[::3] = rng.uniform(0.0, 0.9, e[::3].shape[0])
    ang = [rng.random(n) * 2 * math.pi for _ in range(3)]
    return diskgen.elements_to_state(d.a, e, d.inc, *ang)


def close(x, ref, tol):
    return float(np.abs(x - ref).max() / np.abs(ref).max()) < tol


@pytest.mark.parametrize("n,dt", [(5000, None), (4099, 0.37), (777, 25.0)])
def test_matches_oracle(ctx, orc, n, dt):
    x0, v0 = states(n, seed=n)
    dt = ctx.params.dt_soft if dt is None else dt
    mu = ctx.params.G * ctx.params.m_star
    xr, vr, ok, itr = kepler_drift(x0, v0, mu, dt)
    assert ok.all()
    pos, vel = T(x0), T(v0)
    nu, it = ctx.kepler_drift(pos, vel, dt, iters=True)
    torch.cuda.synchronize()
    assert nu == 0
    x, v = pos.cpu().numpy(), vel.cpu().numpy()
    print(f"n={n} dt={dt}: pos {np.abs(x - xr).max() / np.abs(xr).max():.2e} "
          f"vel {np.abs(v - vr).max() / np.abs(vr).max():.2e} iters max {int(it.max())}")
    assert close(x, xr, 1e-12) and close(v, vr, 1e-12)
    assert np.abs(it.cpu().numpy() - itr).max() <= 1


def test_list_moves_only_its_particles(ctx):
    n = 3000
    x0, v0 = states(n, seed=7)
    idx = np.sort(np.random.default_rng(8).choice(n, size=1111, replace=False)).astype(np.int32)
    mu = ctx.params.G * ctx.params.m_star
    dt = ctx.params.dt_soft
    xr, vr, _, _ = kepler_drift(x0[:, idx], v0[:, idx], mu, dt)
    pos, vel = T(x0), T(v0)
    nu, it = ctx.kepler_drift(pos, vel, dt, index=T(idx, torch.int32), iters=True)
    assert nu == 0 and int(it.min()) >= 1
    x, v = pos.cpu().numpy(), vel.cpu().numpy()
    rest = np.setdiff1d(np.arange(n), idx)
    assert np.array_equal(x[:, rest], x0[:, rest]) and np.array_equal(v[:, rest], v0[:, rest])
    assert close(x[:, idx], xr, 1e-12) and close(v[:, idx], vr, 1e-12)


def test_unbound_and_degenerate_states_are_left_alone(ctx):
    x0, v0 = states(300, seed=9)
    r = np.sqrt((x0 * x0).sum(0))
    v0[:, 3] *= 1.6 * np.sqrt(2.0 / r[3]) / np.sqrt((v0[:, 3] ** 2).sum())  # above escape speed
    v0[:, 100] *= 3.0 * np.sqrt(2.0 / r[100]) / np.sqrt((v0[:, 100] ** 2).sum())
    x0[:, 299] = 0.0  # at the star
    mu = ctx.params.G * ctx.params.m_star
    xr, vr, ok, _ = kepler_drift(x0, v0, mu, 0.3)
    pos, vel = T(x0), T(v0)
    nu, it = ctx.kepler_drift(pos, vel, 0.3, iters=True)
    it = it.cpu().numpy()
    assert list(np.flatnonzero(~ok)) == [3, 100, 299] and nu == 3
    assert (it[~ok] == -1).all() and (it[ok] >= 1).all()
    x, v = pos.cpu().numpy(), vel.cpu().numpy()
    assert np.array_equal(x[:, ~ok], x0[:, ~ok]) and np.array_equal(v[:, ~ok], v0[:, ~ok])
    assert close(x[:, ok], xr[:, ok], 1e-12) and close(v[:, ok], vr[:, ok], 1e-12)


def test_empty_and_bad_lists(ctx, gpu):
    x0, v0 = states(64, seed=10)
    pos, vel = T(x0), T(v0)
    nu, it = ctx.kepler_drift(pos, vel, index=torch.empty(0, dtype=torch.int32, device=DEV), iters=True)
    assert nu == 0 and it.numel() == 0
    assert np.array_equal(pos.cpu().numpy(), x0)
    idx = T(np.array([5, 64, 7], dtype=np.int32), torch.int32)
    with pytest.raises(RuntimeError):
        ctx.kepler_drift(pos, vel, index=idx)
    # the entries in range were drifted, the one out of range skipped
    x = pos.cpu().numpy()
    assert not np.array_equal(x[:, 5], x0[:, 5]) and not np.array_equal(x[:, 7], x0[:, 7])
    assert np.array_equal(np.delete(x, [5, 7], axis=1), np.delete(x0, [5, 7], axis=1))


def test_full_size_disk_sampled(ctx):
    d = diskgen.workload("disk1m_masslaw")
    mu = ctx.params.G * ctx.params.m_star
    dt = ctx.params.dt_soft
    pos, vel = T(d.pos), T(d.vel)
    nu, _ = ctx.kepler_drift(pos, vel, dt)
    assert nu == 0
    s = diskgen.sample_indices(d.n, 20000, seed=12)
    xr, vr, ok, _ = kepler_drift(d.pos[:, s], d.vel[:, s], mu, dt)
    assert ok.all()
    x, v = pos.cpu().numpy()[:, s], vel.cpu().numpy()[:, s]
    assert close(x, xr, 1e-12) and close(v, vr, 1e-12)


# ------------------------------------------------------------- in the hard part
def gparams(gpu, orc, **kw):
    p = orc.Params()
    gp = gpu.Params.defaults().replace(
        G=p.G, m_star=p.m_star, gamma=p.gamma, r_cut0=p.r_cut0, r_cut1=p.r_cut1, r_search0=p.r_search0,
        r_search1=p.r_search1, r_search2=p.r_search2, r_search3=p.r_search3, dt_soft=p.dt_soft, eta=p.eta,
        eta0=p.eta0, hill_length=p.hill_length, vran_bins=p.vran_bins, vran_min_count=p.vran_min_count, k_max=p.k_max,
        theta=0.5, multipole=2)
    return gp.replace(**kw)


def hard(gpu, orc, d, isolated, overlap):
    """One hard part from the disk's state after a soft evaluation; returns
    (pos, vel, dt_hard, labels) on the host."""
    ctx = gpu.Context(gparams(gpu, orc, isolated=isolated, precision=1))
    pos, vel, m = T(d.pos), T(d.vel), T(d.mass)
    ro, rs, _ = ctx.compute_cutoffs(pos, vel, m)
    ctx.build_tree(pos, vel, m, ro, rs)
    ctx.compute_soft_force()
    _, _, lab = ctx.neighbour_list(labels=True)
    dth = torch.zeros_like(m)
    if overlap:
        steps = torch.zeros(d.n, dtype=torch.int32, device=DEV)
        ctx.hard_evaluate(pos, vel, m, ro, dth, steps, ro, rs, slow_log2=3)
    else:
        ctx.hard_step(pos, vel, m, ro, dt_hard=dth)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    out = pos.cpu().numpy(), vel.cpu().numpy(), dth.cpu().numpy(), lab.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("overlap", [False, True])
def test_isolated_particles_take_the_kepler_drift(gpu, orc, overlap):
    """isolated = 1: the clusters of one member move exactly on their orbits
    (the oracle's drift), every other cluster exactly as with isolated = 0
    (bit for bit: the same Hermite kernels on the same clusters)."""
    d = diskgen.workload("disk64k_masslaw")
    x1, v1, h1, lab = hard(gpu, orc, d, 1, overlap)
    x0, v0, h0, lab0 = hard(gpu, orc, d, 0, overlap)
    assert np.array_equal(lab, lab0)
    single = np.bincount(lab, minlength=d.n)[lab] == 1
    print(f"overlap={overlap}: {int(single.sum())} of {d.n} particles isolated")
    assert 0 < single.sum() < d.n
    rest = ~single
    assert np.array_equal(x1[:, rest], x0[:, rest]) and np.array_equal(v1[:, rest], v0[:, rest])
    assert np.array_equal(h1[rest], h0[rest]) and (h1[single] == 0.0).all()
    p = orc.Params()
    xr, vr, ok, _ = kepler_drift(d.pos[:, single], d.vel[:, single], p.G * p.m_star, p.dt_soft)
    assert ok.all()
    assert close(x1[:, single], xr, 1e-12) and close(v1[:, single], vr, 1e-12)
    # and the Hermite steps of the isolated particles agree with the exact
    # drift to the integrator's accuracy
    assert close(x0[:, single], xr, 1e-7)
