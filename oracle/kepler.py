"""Oracle Kepler drift of isolated particles (TEST INFRASTRUCTURE ONLY).

Section 2.2 lets a particle without neighbours move on the two-body orbit
about the star over the soft step (the paper solves Kepler's equation by
Newton-Raphson for these particles).  Plain FP64 numpy, particle by particle
in vector form, written from the two-body solution in the difference of the
eccentric anomaly dE (the f and g functions):

    mu = G M_*, r0 = |x0|, 1/a = 2/r0 - |v0|^2/mu (bound orbits: a > 0),
    n = sqrt(mu / a^3), ec = 1 - r0/a (= e cos E0), es = x0.v0 / sqrt(mu a)
    (= e sin E0);
    Kepler's equation for dE:  dE - ec sin dE + es (1 - cos dE) = n dt,
    solved by Newton-Raphson from dE = n dt;
    r = a (1 - ec cos dE + es sin dE),
    f = 1 - (a/r0)(1 - cos dE),        g = dt + (sin dE - dE)/n,
    fd = -a^2 n sin dE / (r r0),       gd = 1 - (a/r)(1 - cos dE),
    x = f x0 + g v0,  v = fd x0 + gd v0.

States that are not on a bound orbit (1/a <= 0, or 1/a not finite as at the
star's own position) are returned unchanged and reported in the mask.
"""
from __future__ import annotations

import numpy as np


def kepler_drift(pos, vel, mu: float, dt: float, tol: float = 1e-15, max_iter: int = 50):
    """(pos (3, n), vel (3, n), bound (n,) bool, iterations (n,)) after dt."""
    x0 = np.asarray(pos, dtype=np.float64)
    v0 = np.asarray(vel, dtype=np.float64)
    r0 = np.sqrt((x0 * x0).sum(0))
    v2 = (v0 * v0).sum(0)
    with np.errstate(all="ignore"):  # states off a bound orbit are masked out below
        return _drift(x0, v0, r0, v2, mu, dt, tol, max_iter)


def _drift(x0, v0, r0, v2, mu, dt, tol, max_iter):
    inv_a = 2.0 / r0 - v2 / mu
    bound = (inv_a > 0.0) & np.isfinite(inv_a)
    a = np.where(bound, 1.0 / np.where(bound, inv_a, 1.0), 1.0)
    n = np.sqrt(mu / a ** 3)
    ec = 1.0 - r0 / a
    es = (x0 * v0).sum(0) / np.sqrt(mu * a)
    M = n * dt
    dE = M.copy()
    iters = np.zeros(x0.shape[1], dtype=np.int64)
    active = bound.copy()
    for _ in range(max_iter):
        if not active.any():
            break
        F = dE - ec * np.sin(dE) + es * (1.0 - np.cos(dE)) - M
        Fp = 1.0 - ec * np.cos(dE) + es * np.sin(dE)
        step = np.where(active, F / Fp, 0.0)
        dE = dE - step
        iters += active
        active = active & (np.abs(step) > tol * np.maximum(1.0, np.abs(dE)))
    c, s = np.cos(dE), np.sin(dE)
    r = a * (1.0 - ec * c + es * s)
    f = 1.0 - (a / r0) * (1.0 - c)
    g = dt + (s - dE) / n
    fd = -a * a * n * s / (r * r0)
    gd = 1.0 - (a / r) * (1.0 - c)
    x = np.where(bound, f * x0 + g * v0, x0)
    v = np.where(bound, fd * x0 + gd * v0, v0)
    return x, v, bound, iters
