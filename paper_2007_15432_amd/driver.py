"""The P3T soft step (Section 2.2, steps (2)-(8) without collisions) as a
sequence of library calls.  Orchestration only: every numerical step runs in
libp3t's kernels.

    init:  cut-off radii; tree; soft force a_soft and neighbour lists  (2)
    step:  v += a_soft dt/2                                           (3)
           neighbour clusters from the lists of the last evaluation   (4)
           Hermite integration of every cluster over dt               (5)
           ((4)-(5) in one library call, p3t_hard_step, by default)
           tree; soft force and neighbour lists at the new state      (7)
           v += a_soft dt/2                                           (8)

The cut-off radii are fixed between collisions (Section 2.4: they are
recomputed after a merger); `recompute_cutoffs` recomputes them every step
instead (used to time the cut-off stage as part of the step).
"""
from __future__ import annotations

import torch

from .api import Context, Params


class P3TStepper:
    """graph=True evaluates tree + force through p3t_evaluate's captured
    hipGraph (replayed every step: positions, masses, radii and the
    acceleration live in fixed buffers)."""

    def __init__(self, ctx: Context, pos, vel, mass, recompute_cutoffs: bool = False, graph: bool = False,
                 fused_hard: bool = True):
        self.ctx = ctx
        self.graph = graph
        self.fused_hard = fused_hard
        self.pos, self.vel, self.mass = pos, vel, mass
        self.n = int(mass.shape[0])
        self.dt = ctx.params.dt_soft
        self.recompute = recompute_cutoffs
        self.r_out, self.r_search, self.v_ran = ctx.compute_cutoffs(pos, vel, mass)
        self.dt_hard = torch.zeros(self.n, dtype=torch.float64, device=pos.device)
        self.acc = torch.empty((3, self.n), dtype=torch.float64, device=pos.device)
        self.n_clusters = 0
        self._evaluate()

    def _evaluate(self):
        c = self.ctx
        if self.graph:
            c.evaluate(self.pos, self.vel, self.mass, self.r_out, self.r_search, out=self.acc, graph=True)
        else:
            c.build_tree(self.pos, self.vel, self.mass, self.r_out, self.r_search)
            c.compute_soft_force(out=self.acc)
        if not self.fused_hard:
            self.row_ptr, self.col, self.label = c.neighbour_list(labels=True)

    @property
    def last(self) -> dict:
        """Counters of the last evaluation (synchronises)."""
        return self.ctx.stats()

    def step(self):
        c = self.ctx
        c.kick(self.acc, self.vel, 0.5 * self.dt)
        if self.fused_hard:
            self.n_clusters = c.hard_step(self.pos, self.vel, self.mass, self.r_out, dt_hard=self.dt_hard)
        else:
            cl_ptr, members = c.clusters(self.label)
            self.n_clusters = int(cl_ptr.shape[0]) - 1
            c.hermite_cluster_step(self.pos, self.vel, self.mass, self.r_out, cl_ptr, members, dt_hard=self.dt_hard,
                                   energy=False)
        if self.recompute:
            c.compute_cutoffs(self.pos, self.vel, self.mass, out=(self.r_out, self.r_search, self.v_ran))
        self._evaluate()
        c.kick(self.acc, self.vel, 0.5 * self.dt)

    def interactions(self) -> int:
        s = self.last
        return int(s["n_near"] + s["n_far"] + s["n_cell"])


__all__ = ["P3TStepper", "Params"]
