"""Pins for the oracle's neighbour test (Section 2.3: eq. (rsearch), eq.
(rsearch1), the t_min cases and the slow-pair clause).

The oracle decides with a fixed division- and root-free FP64 sequence.  It is
pinned here against the literal definition evaluated in exact rational
arithmetic (Fractions): candidate r < max(r_search,i, r_search,j); closest
approach |r_ij + v_ij t_min| with t_min = clamp(-r.v/v^2, 0, dt) compared
with Rsearch2 r_out,ij; slow pairs |v_ij| < Rsearch3 G (m_i+m_j)/r^2 dt/2.
The only allowed disagreements are pairs whose exact margin to a threshold is
below FP64 resolution (counted, must be rare).  Also: symmetry of the
relation and hand-built cases for every branch.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import diskgen


def exact_neighbour(pi, pj, p):
    """Literal definition in exact arithmetic.  Returns (decision, margin)
    where margin is the smallest relative distance of any deciding quantity
    from its threshold."""
    xi, xj = [Fr(float(v)) for v in pi], [Fr(float(v)) for v in pj]
    d = [xi[k] - xj[k] for k in range(3)]
    u = [xi[3 + k] - xj[3 + k] for k in range(3)]
    rr = sum(c * c for c in d)
    rs = max(xi[8], xj[8])
    margins = []
    margins.append(abs(rr - rs * rs) / (rs * rs))
    if not rr < rs * rs:
        return False, min(margins)
    vv = sum(c * c for c in u)
    rv = sum(d[k] * u[k] for k in range(3))
    dt = Fr(p.dt_soft)
    if vv == 0:
        tmin = Fr(0)
    else:
        tmin = min(max(-rv / vv, Fr(0)), dt)
    dmin2 = sum((d[k] + u[k] * tmin) ** 2 for k in range(3))
    R = Fr(p.r_search2) * max(xi[7], xj[7])
    close = dmin2 <= R * R
    margins.append(abs(dmin2 - R * R) / (R * R))
    A = Fr(p.r_search3) * Fr(p.G) * (xi[6] + xj[6]) / rr * dt / 2  # a_ij dt R3 / 2
    slow = vv < A * A
    if A > 0:
        margins.append(abs(vv - A * A) / (A * A))
    return close or slow, min(margins)


def _pairs_from_ring(orc, p, n=1024, seed=11):
    d = diskgen.dense_ring(n, seed=seed)
    ro, rs, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
    return d, ro, rs


def test_predicate_matches_exact_definition(orc):
    p = orc.Params(r_cut0=10.0)
    d, ro, rs = _pairs_from_ring(orc, p)
    X = np.vstack([d.pos, d.vel, d.mass[None], ro[None], rs[None]])  # (9, n)
    rng = np.random.default_rng(5)
    # candidate-rich sample: nearest pairs by position plus random pairs
    from scipy.spatial import cKDTree

    tr = cKDTree(d.pos.T)
    pairs = list(tr.query_pairs(float(rs.max()) * 1.5))
    pairs = pairs[:3000] + [tuple(rng.integers(0, d.n, 2)) for _ in range(500)]
    n_tight = n_agree = 0
    branches = set()
    for i, j in pairs:
        if i == j:
            continue
        ex, margin = exact_neighbour(X[:, i], X[:, j], p)
        got = orc.is_neighbour(X[:, i], X[:, j], p)
        if margin < 1e-12:
            n_tight += 1
            continue
        assert got == ex, (i, j)
        n_agree += 1
        # which t_min branch (for coverage)
        dd = X[:3, i] - X[:3, j]
        uu = X[3:6, i] - X[3:6, j]
        if np.dot(dd, dd) < max(rs[i], rs[j]) ** 2:
            vv, rv = np.dot(uu, uu), np.dot(dd, uu)
            branches.add("t0" if (vv == 0 or rv >= 0) else ("interior" if -rv < p.dt_soft * vv else "tdt"))
    assert n_agree > 2000 and n_tight <= 2
    assert branches == {"t0", "interior", "tdt"}


def test_relation_is_symmetric(orc):
    p = orc.Params(r_cut0=10.0)
    d, ro, rs = _pairs_from_ring(orc, p)
    row_ptr, col = orc.neighbour_rows(d.pos, d.vel, d.mass, ro, rs, p)
    pairs = set()
    for i in range(d.n):
        for j in col[row_ptr[i]:row_ptr[i + 1]]:
            pairs.add((i, int(j)))
    assert len(pairs) > 1000
    assert all((j, i) in pairs for (i, j) in pairs)
    # rows ascending, no self
    for i in range(d.n):
        r = col[row_ptr[i]:row_ptr[i + 1]]
        assert np.all(np.diff(r) > 0) and i not in r


def _pt(x, v, m=1e-9, ro=1e-3, rs=2e-3):
    return np.array([x[0], x[1], x[2], v[0], v[1], v[2], m, ro, rs])


def test_hand_cases(orc):
    p = orc.Params(r_search2=1.0, r_search3=0.0)  # plain closest-approach test
    dt = p.dt_soft
    o = _pt([1, 0, 0], [0, 0, 0])
    # beyond the search radius: never a neighbour
    assert not orc.is_neighbour(o, _pt([1 + 2.5e-3, 0, 0], [0, 0, 0]), p)
    # at rest, inside r_out: neighbour (t_min = 0)
    assert orc.is_neighbour(o, _pt([1 + 0.9e-3, 0, 0], [0, 0, 0]), p)
    # at rest, between r_out and r_search: excluded
    assert not orc.is_neighbour(o, _pt([1 + 1.5e-3, 0, 0], [0, 0, 0]), p)
    # receding from 1.5 r_out: excluded (t_min = 0)
    assert not orc.is_neighbour(o, _pt([1 + 1.5e-3, 0, 0], [1e-3, 0, 0]), p)
    # approaching, passes through within the step with offset 0.5 r_out (interior minimum)
    vfast = 1.0e-1
    assert orc.is_neighbour(o, _pt([1 + 1.9e-3, 0.5e-3, 0], [-vfast, 0, 0]), p)
    # approaching on a parallel track with offset 1.5 r_out: excluded
    assert not orc.is_neighbour(o, _pt([1 + 1.9e-3, 1.5e-3, 0], [-vfast, 0, 0]), p)
    # approaching slowly: reaches 1.9e-3 - v dt at the end of the step (t_min = dt)
    vslow = 0.95e-3 / dt
    assert orc.is_neighbour(o, _pt([1 + 1.9e-3, 0, 0], [-vslow, 0, 0]), p)
    vslow2 = 0.85e-3 / dt
    assert not orc.is_neighbour(o, _pt([1 + 1.9e-3, 0, 0], [-vslow2, 0, 0]), p)
    # slow-pair clause keeps a receding pair with |v| < R3 a_ij dt / 2
    p3 = orc.Params(r_search2=1.0, r_search3=2.0)
    r = 1.5e-3
    a = 2e-9 / r**2
    vkeep = 0.9 * 2.0 * a * dt / 2
    assert orc.is_neighbour(o, _pt([1 + r, 0, 0], [vkeep, 0, 0]), p3)
    assert not orc.is_neighbour(o, _pt([1 + r, 0, 0], [1.2 * 2.0 * a * dt / 2, 0, 0]), p3)


def test_pair_search_radius_is_the_larger(orc):
    p = orc.Params(r_search2=1.0, r_search3=0.0)
    a = _pt([1, 0, 0], [0, 0, 0], ro=1e-3, rs=1e-3)
    b = _pt([1 + 1.5e-3, 0, 0], [-1e-2, 0, 0], ro=1e-3, rs=3e-3)  # only b's radius covers the pair
    assert orc.is_neighbour(a, b, p) and orc.is_neighbour(b, a, p)


def test_subset_rows_match_full(orc):
    p = orc.Params(r_cut0=10.0)
    d, ro, rs = _pairs_from_ring(orc, p, n=512)
    rp, col = orc.neighbour_rows(d.pos, d.vel, d.mass, ro, rs, p)
    idx = np.array([3, 100, 511, 0])
    rp2, col2 = orc.neighbour_rows(d.pos, d.vel, d.mass, ro, rs, p, idx=idx)
    for k, i in enumerate(idx):
        assert np.array_equal(col2[rp2[k]:rp2[k + 1]], col[rp[i]:rp[i + 1]])
