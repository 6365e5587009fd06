"""Oracle leapfrog and its adjoint (TEST INFRASTRUCTURE ONLY).

Plain FP64 numpy around the C oracle: kick-drift-kick steps whose soft kicks
use the direct soft force (eq. (softforce)) with fixed pair cut-offs and
whose star kick and drift are written out; the reverse pass walks the steps
backwards with the oracle's soft-force vector-Jacobian product and the
analytic Jacobian of the star's acceleration,
    d(-GM x / r^3)/dx = -GM (I / r^3 - 3 x x^T / r^5)  (symmetric).
No blocking, no checkpointing: every state is stored.
"""
from __future__ import annotations

import numpy as np

from . import Params, soft_acc, soft_adjoint


def star_acc(x, GM=1.0):
    r2 = (x * x).sum(0)
    return -GM * x / (r2 * np.sqrt(r2))


def star_vjp(x, lam, GM=1.0):
    """lam . d(star_acc)/dx, per particle."""
    r2 = (x * x).sum(0)
    r = np.sqrt(r2)
    xl = (x * lam).sum(0)
    return -GM * (lam / (r2 * r) - 3.0 * x * xl / (r2 * r2 * r))


def leapfrog(x, v, m, r_out, p: Params, h, n_steps, GM=1.0):
    """Returns (x, v) after n_steps, and the tape of states for the adjoint."""
    tape = []
    x, v = x.copy(), v.copy()
    for _ in range(n_steps):
        x0 = x
        v = v + 0.5 * h * soft_acc(x0, m, r_out, p)
        v = v + 0.5 * h * star_acc(x0, GM)
        x = x0 + h * v
        v = v + 0.5 * h * star_acc(x, GM)
        v = v + 0.5 * h * soft_acc(x, m, r_out, p)
        tape.append((x0, x))
    return x, v, tape


def leapfrog_adjoint(m, r_out, p: Params, h, tape, lx, lv, GM=1.0):
    """Given the cotangents (lx, lv) of the final (x, v), returns the
    cotangents of the initial (x, v) and of the masses."""
    lx, lv = lx.copy(), lv.copy()
    lm = np.zeros_like(m)
    for x0, x1 in reversed(tape):
        # v4 = v3 + h/2 a_soft(x1)
        gx, gm = soft_adjoint(x1, m, r_out, lv, p)
        lx += 0.5 * h * gx
        lm += 0.5 * h * gm
        # v3 = v2 + h/2 a_star(x1)
        lx += 0.5 * h * star_vjp(x1, lv, GM)
        # x1 = x0 + h v2
        lv = lv + h * lx
        # v2 = v1 + h/2 a_star(x0);  v1 = v0 + h/2 a_soft(x0)
        lx = lx + 0.5 * h * star_vjp(x0, lv, GM)
        gx, gm = soft_adjoint(x0, m, r_out, lv, p)
        lx += 0.5 * h * gx
        lm += 0.5 * h * gm
    return lx, lv, lm
