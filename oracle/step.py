"""Oracle P3T soft step (TEST INFRASTRUCTURE ONLY).

One step of the time-integration procedure of Section 2.2, steps (2)-(8)
without collisions, i.e. the splitting of eq. (HamiltonSol): a half kick by
the soft force, the hard part over the soft step, a new soft force at the
new state, a second half kick.  Plain FP64 around the oracle's direct
functions, in the paper's order:

  (2) a_soft(x) by the direct sum of eq. (softforce) with the pair cut-off
      of eq. (rout2); the neighbour rows of Section 2.3 at (x, v);
  (3) v += a_soft dt / 2;
  (4) neighbour clusters from those rows: label = minimum index of the
      connected component (Section 2.3), members sorted by (label, index);
  (5) every cluster integrated over dt: the fourth-order Hermite oracle
      with the star and the (1 - K) pair forces (eq. (hardforce)); with
      isolated = 1 the clusters of one member (particles without
      neighbours) move on their Kepler orbits instead (Section 2.2, step
      (5)(ii)) and carry no hard step;
  (7) a_soft and the neighbour rows again, at the new state;
  (8) v += a_soft dt / 2.

The cut-off and search radii stay fixed (they change only after a
collision, step (9)).  No blocking, no reordering: every stage is one call.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import Params, cluster_csr, cutoffs, hermite_clusters, hermite_collide, labels, neighbour_rows, soft_acc
from .kepler import kepler_drift


@dataclass
class StepState:
    """State carried between steps: positions, velocities, the soft force
    and neighbour rows of the last evaluation, each particle's hard step."""

    pos: np.ndarray
    vel: np.ndarray
    acc: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    dt_hard: np.ndarray
    steps: np.ndarray | None = None  # block steps of each particle's cluster in the last hard part
    n_clusters: int = 0
    hermite_status: int = 0


def evaluate(pos, vel, mass, r_out, r_search, p: Params):
    """Step (2) / (7): soft acceleration and neighbour rows at (pos, vel)."""
    acc = soft_acc(pos, mass, r_out, p)
    rp, col = neighbour_rows(pos, vel, mass, r_out, r_search, p)
    return acc, rp, col


def init(pos, vel, mass, r_out, r_search, p: Params) -> StepState:
    """Steps (1)-(2): the first evaluation."""
    pos = np.array(pos, dtype=np.float64, order="C")
    vel = np.array(vel, dtype=np.float64, order="C")
    acc, rp, col = evaluate(pos, vel, mass, r_out, r_search, p)
    return StepState(pos, vel, acc, rp, col, np.zeros(pos.shape[1]))


def hard_part(pos, vel, mass, r_out, row_ptr, col, dt_hard, p: Params, isolated: int = 0):
    """Steps (4)-(5): clusters from the neighbour rows, each integrated over
    dt_soft.  Returns (pos, vel, n_clusters, status, steps) with steps the
    block-step count of each particle's cluster (1 for a Kepler drift);
    dt_hard is updated in place."""
    lab, _ = labels(row_ptr, col)
    cl_ptr, members = cluster_csr(lab)
    nc = cl_ptr.shape[0] - 1
    sizes = np.diff(cl_ptr)
    pos, vel = pos.copy(), vel.copy()
    steps = np.zeros(pos.shape[1], dtype=np.int64)
    if isolated:
        single = members[cl_ptr[:-1][sizes == 1]]
        multi = np.flatnonzero(sizes > 1)
        # the clusters of several members, in their own CSR
        m_ptr = np.zeros(multi.shape[0] + 1, dtype=np.int32)
        m_ptr[1:] = np.cumsum(sizes[multi])
        m_mem = np.concatenate([members[cl_ptr[c]:cl_ptr[c + 1]] for c in multi]) if multi.size else \
            np.zeros(0, dtype=np.int32)
        xs, vs, bound, _ = kepler_drift(pos[:, single], vel[:, single], p.G * p.m_star, p.dt_soft)
        if not bound.all():
            raise FloatingPointError("an isolated particle is not on a bound orbit")
        status = 0
        if multi.size:
            pos, vel, _, _, ns, status = hermite_clusters(pos, vel, mass, r_out, m_ptr, m_mem, p, dt_hard=dt_hard)
            steps[m_mem] = np.repeat(ns, np.diff(m_ptr))
        pos[:, single] = xs
        vel[:, single] = vs
        dt_hard[single] = 0.0
        steps[single] = 1
    else:
        pos, vel, _, _, ns, status = hermite_clusters(pos, vel, mass, r_out, cl_ptr, members, p, dt_hard=dt_hard)
        steps[members] = np.repeat(ns, sizes)
    return pos, vel, nc, status, steps


def step(s: StepState, mass, r_out, r_search, p: Params, isolated: int = 0) -> StepState:
    """Steps (3)-(8) from the state of the last evaluation; returns the new
    state (the input is not modified)."""
    h = 0.5 * p.dt_soft
    vel = s.vel + h * s.acc                                             # (3)
    dt_hard = s.dt_hard.copy()
    pos, vel, nc, status, steps = hard_part(s.pos, vel, mass, r_out, s.row_ptr, s.col, dt_hard, p, isolated)  # (4)-(5)
    acc, rp, col = evaluate(pos, vel, mass, r_out, r_search, p)        # (7)
    vel = vel + h * acc                                                 # (8)
    return StepState(pos, vel, acc, rp, col, dt_hard, steps, nc, status)


def run(pos, vel, mass, r_out, r_search, p: Params, n_steps: int, isolated: int = 0):
    """n_steps steps from an initial state; returns the list of states
    (the initial evaluation first)."""
    s = init(pos, vel, mass, r_out, r_search, p)
    out = [s]
    for _ in range(n_steps):
        s = step(s, mass, r_out, r_search, p, isolated)
        out.append(s)
    return out


def total_energy(pos, vel, mass, p: Params) -> float:
    """H_soft + H_hard of eq. (soft) and eq. (hard) over all particles.  The
    changeover weights add up to one for every pair (W + (1 - W)), so the sum
    is the Newtonian energy of the planetesimals about a fixed star; it is
    written here directly as that plain definition."""
    x = np.asarray(pos, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64)
    kin = 0.5 * float((m * (v * v).sum(0)).sum())
    star = -p.G * p.m_star * float((m / np.sqrt((x * x).sum(0))).sum())
    pair = 0.0
    n = m.shape[0]
    for i in range(n - 1):
        d = x[:, i + 1:] - x[:, i:i + 1]
        r = np.sqrt((d * d).sum(0))
        pair -= p.G * m[i] * float((m[i + 1:] / r).sum())
    return kin + star + pair


# -- perfect-accretion collisions (Section 2.5.1) --------------------------------
def merge_bodies(pos, vel, mass, dt_hard, merged_into):
    """Each composite left by the hard part becomes one particle: the one at
    its lowest index keeps the (shared) state and takes the total mass
    (summed in index order); the others are removed.  Returns (pos, vel,
    mass, dt_hard, keep) with keep the mask of the surviving indices."""
    n = mass.shape[0]
    merged_into = np.asarray(merged_into)
    keep = merged_into == np.arange(n)
    total = np.zeros(n)
    for g in range(n):  # index order
        total[merged_into[g]] += mass[g]
    return (np.ascontiguousarray(pos[:, keep]), np.ascontiguousarray(vel[:, keep]), total[keep],
            np.ascontiguousarray(dt_hard[keep]), keep)


def step_collide(s: StepState, mass, r_out, r_search, p: Params, f: float, rho: float, isolated: int = 1):
    """One soft step with perfect accretion: kick, hard part with collision
    detection in every cluster (composites move as one body), then, if any
    merger happened, the composites become single particles and the cut-off
    and search radii of all particles are recomputed (step (9)); the soft
    force and neighbour rows of the resulting system, the second kick.
    Reading: the merger is applied before the evaluation of step (7) rather
    than after the kick of step (8), so one evaluation serves both the second
    kick and the next step; the kick of a merged body uses its own soft force
    (no averaging of the two parts' soft forces, hence no E_disp,Soft).
    Returns (state, mass, r_out, r_search, eps (6,) summed over the mergers,
    number of particles removed)."""
    h = 0.5 * p.dt_soft
    vel = s.vel + h * s.acc
    dt_hard = s.dt_hard.copy()
    lab, _ = labels(s.row_ptr, s.col)
    cl_ptr, members = cluster_csr(lab)
    sizes = np.diff(cl_ptr)
    pos = s.pos.copy()
    n = pos.shape[1]
    merged = np.arange(n, dtype=np.int32)
    eps = np.zeros(6)
    status = 0
    steps = np.zeros(n, dtype=np.int64)
    single = members[cl_ptr[:-1][sizes == 1]] if isolated else np.zeros(0, dtype=np.int32)
    multi = np.flatnonzero(sizes > 1) if isolated else np.arange(sizes.shape[0])
    if multi.size:
        m_ptr = np.zeros(multi.shape[0] + 1, dtype=np.int32)
        m_ptr[1:] = np.cumsum(sizes[multi])
        m_mem = np.concatenate([members[cl_ptr[c]:cl_ptr[c + 1]] for c in multi]).astype(np.int32)
        r = hermite_collide(pos, vel, mass, r_out, m_ptr, m_mem, p, f, rho, dt_hard=dt_hard)
        pos, vel, status = r["pos"], r["vel"], r["status"]
        merged[m_mem] = r["merged_into"][m_mem]
        eps = r["eps"].sum(axis=0)
        steps[m_mem] = np.repeat(r["nsteps"], np.diff(m_ptr))
    if single.size:
        xs, vs, bound, _ = kepler_drift(pos[:, single], vel[:, single], p.G * p.m_star, p.dt_soft)
        if not bound.all():
            raise FloatingPointError("an isolated particle is not on a bound orbit")
        pos[:, single] = xs
        vel[:, single] = vs
        dt_hard[single] = 0.0
        steps[single] = 1
    removed = 0
    mass = np.asarray(mass, dtype=np.float64)
    if np.any(merged != np.arange(n)):
        pos, vel, mass, dt_hard, keep = merge_bodies(pos, vel, mass, dt_hard, merged)
        steps = steps[keep]
        removed = int(n - keep.sum())
        r_out, r_search, _ = cutoffs(pos, vel, mass, p)
    acc, rp, col = evaluate(pos, vel, mass, r_out, r_search, p)
    vel = vel + h * acc
    return StepState(pos, vel, acc, rp, col, dt_hard, steps, int(sizes.shape[0]), status), mass, r_out, r_search, \
        eps, removed
