"""Pins for the oracle's neighbour-cluster labels (Section 2.3 steps i-iii)
and its block-step Hermite integrator (Section 2.1.1, step (5) of Section 2.2).

Labels: the fixed point of the min-propagation is, by definition, the minimum
index of each connected component of the neighbour graph; pinned against
scipy's connected components and hand-built graphs (a chain whose minimum
sits at one end needs the most sweeps, the paper's a..g example converges to
the smallest index a).

Hermite: pinned against the analytic two-body (Kepler) solution, fourth-order
convergence (the error falls ~16x when the Aarseth steps halve), conservation
of the hard-part energy eq. (hard) for bound pairs inside the changeover
region, and the batch driver against single-cluster calls.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import diskgen


def _csr_from_edges(n, edges):
    rows = [[] for _ in range(n)]
    for i, j in edges:
        rows[i].append(j)
        rows[j].append(i)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = []
    for i in range(n):
        r = sorted(set(rows[i]))
        col += r
        row_ptr[i + 1] = row_ptr[i] + len(r)
    return row_ptr, np.array(col, dtype=np.int32)


def _cc_min_labels(row_ptr, col):
    n = len(row_ptr) - 1
    g = csr_matrix((np.ones(len(col)), col, row_ptr), shape=(n, n))
    nc, comp = connected_components(g, directed=False)
    mins = np.full(nc, n)
    for i in range(n):
        mins[comp[i]] = min(mins[comp[i]], i)
    return mins[comp]


def test_labels_random_graphs(orc):
    rng = np.random.default_rng(0)
    for n, ne in [(1, 0), (10, 0), (200, 150), (1000, 900), (500, 2000)]:
        edges = [tuple(rng.integers(0, n, 2)) for _ in range(ne)]
        edges = [(i, j) for i, j in edges if i != j]
        rp, col = _csr_from_edges(n, edges)
        lab, _ = orc.labels(rp, col)
        assert np.array_equal(lab, _cc_min_labels(rp, col))


def test_labels_chain_and_example(orc):
    n = 50
    perm = np.arange(n)[::-1]  # chain 49-48-...-0: minimum at the far end
    rp, col = _csr_from_edges(n, [(perm[k], perm[k + 1]) for k in range(n - 1)])
    lab, sweeps = orc.labels(rp, col)
    assert np.all(lab == 0) and sweeps == n  # n-1 propagating sweeps + 1 confirming
    # a..g (indices 0..6) connected as two chains joined in the middle, plus isolated 7, 8
    rp, col = _csr_from_edges(9, [(6, 5), (5, 2), (2, 3), (3, 0), (4, 1), (1, 3)])
    lab, _ = orc.labels(rp, col)
    assert list(lab) == [0, 0, 0, 0, 0, 0, 0, 7, 8]


def _kepler_state(a, e, M, mu=1.0):
    E = brentq(lambda E: E - e * math.sin(E) - M, M - 1.0, M + 1.0, xtol=1e-15)
    n = math.sqrt(mu / a**3)
    x = a * (math.cos(E) - e)
    y = a * math.sqrt(1 - e * e) * math.sin(E)
    den = 1 - e * math.cos(E)
    vx = -a * n * math.sin(E) / den
    vy = a * n * math.sqrt(1 - e * e) * math.cos(E) / den
    return np.array([[x], [y], [0.0]]), np.array([[vx], [vy], [0.0]])


def _kepler_error(orc, eta, e=0.3, a=1.0, steps=4):
    p = orc.Params(eta=eta, eta0=eta / 10)
    x, v = _kepler_state(a, e, 0.2)
    m = np.array([1e-12])
    ro = np.array([1e-4])
    dt = p.dt_soft
    for _ in range(steps):
        x, v, e0, e1, ns, st = orc.hermite_clusters(x, v, m, ro, np.array([0, 1]), np.array([0]), p)
        assert st == 0
    n = math.sqrt(1.0 / a**3)
    xr, vr = _kepler_state(a, e, 0.2 + n * dt * steps)
    return float(np.abs(x - xr).max()), float(np.abs(v - vr).max())


def test_hermite_kepler_orbit(orc):
    ex, ev = _kepler_error(orc, 0.01)
    assert ex < 1e-7 and ev < 5e-7


def test_hermite_fourth_order(orc):
    """One orbit (e = 0.3) in one call with a negligible start-up step, so the
    Aarseth steps dominate; eta / 4 halves every step under the square root,
    so a fourth-order scheme's error falls ~2^4."""
    errs = []
    for eta in (0.04, 0.01, 0.0025, 0.000625):
        p = orc.Params(eta=eta, eta0=1e-7, dt_soft=2 * math.pi)
        x, v = _kepler_state(1.0, 0.3, 0.2)
        x, v, e0, e1, ns, st = orc.hermite_clusters(x, v, np.array([1e-12]), np.array([1e-4]), np.array([0, 1]),
                                                    np.array([0]), p)
        assert st == 0
        xr, _ = _kepler_state(1.0, 0.3, 0.2 + 2 * math.pi)
        errs.append(float(np.abs(x - xr).max()))
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(11 < r < 22 for r in ratios), (errs, ratios)


def test_hermite_carried_step(orc):
    """A step carried in from the previous soft step replaces the initial
    criterion, and the last step is written back."""
    p = orc.Params(eta=0.01, eta0=0.001)
    x, v = _kepler_state(1.0, 0.1, 0.0)
    m, ro = np.array([1e-12]), np.array([1e-4])
    dh = np.zeros(1)
    x1, v1, _, _, ns1, _ = orc.hermite_clusters(x, v, m, ro, np.array([0, 1]), np.array([0]), p, dt_hard=dh)
    assert dh[0] > 0 and math.log2(p.dt_soft / dh[0]) % 1 == 0
    x2, v2, _, _, ns2, _ = orc.hermite_clusters(x1, v1, m, ro, np.array([0, 1]), np.array([0]), p, dt_hard=dh)
    x3, v3, _, _, ns3, _ = orc.hermite_clusters(x1, v1, m, ro, np.array([0, 1]), np.array([0]), p)
    assert ns2[0] < ns3[0]  # no start-up ramp
    assert np.abs(x2 - x3).max() < 1e-8


def test_hermite_energy_bound_pair_in_changeover(orc):
    """Two planetesimals on nearly identical orbits, separated by ~0.5 r_out,
    so the pair force is split by K for the whole step."""
    x1, v1 = _kepler_state(1.0, 0.0, 0.0)
    x = np.hstack([x1, x1 + np.array([[0.0], [6e-4], [0.0]])])
    v = np.hstack([v1, v1 + np.array([[1e-5], [0.0], [0.0]])])
    m = np.array([1e-8, 1e-8])
    ro = np.array([1.2e-3, 1.0e-3])
    errs = []
    for eta in (0.0025, 0.000625):
        p = orc.Params(eta=eta, eta0=eta / 10)
        xs, vs, e0, e1, ns, st = orc.hermite_clusters(x, v, m, ro, np.array([0, 2]), np.array([0, 1]), p)
        assert st == 0
        errs.append(abs(e1[0] - e0[0]) / abs(e0[0]))
    # the bound pair's energy error falls as eta^2 (dt^4) and is small
    assert errs[0] / errs[1] > 10 and errs[1] < 1e-9, errs
    # the pair interaction is active (the relative motion differs from two
    # independent Kepler orbits)
    xs_free, _, _, _, _, _ = orc.hermite_clusters(x, v, m, ro, np.array([0, 1, 2]), np.array([0, 1]), p)
    assert np.abs(xs - xs_free).max() > 1e-9


def test_hermite_batch_equals_single(orc):
    p = orc.Params(eta=0.02, eta0=0.002)
    d = diskgen.make_disk(4096, 0.5, 1.5, seed=2)
    ro, _, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
    cl = diskgen.hermite_clusters(d, n_clusters=30, seed=4, n_max=24, r_out=ro, compact=0.7)
    xb, vb, e0, e1, ns, st = orc.hermite_clusters(cl["pos"], cl["vel"], cl["mass"], cl["r_out"], cl["cl_ptr"],
                                                  np.arange(cl["pos"].shape[1]), p)
    assert st == 0
    for c in [0, 7, int(np.argmax(cl["sizes"]))]:
        a, b = cl["cl_ptr"][c], cl["cl_ptr"][c + 1]
        xs, vs, f0, f1, nss, st1 = orc.hermite_clusters(
            cl["pos"][:, a:b], cl["vel"][:, a:b], cl["mass"][a:b], cl["r_out"][a:b], np.array([0, b - a]),
            np.arange(b - a), p)
        assert np.array_equal(xs, xb[:, a:b]) and f1[0] == e1[c] and nss[0] == ns[c]
    rel = np.abs(e1 - e0) / np.abs(e0)
    assert np.max(rel) < 1e-4  # compacted clusters at eta = 0.02: bounded, not tiny
