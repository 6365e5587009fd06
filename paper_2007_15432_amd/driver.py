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

The cut-off radii are fixed between collisions (Section 2.2 step (9): they
are recomputed after a merger).  `monitor_cutoffs` computes the radii of the
current state every step into buffers of their own (r_out_now, r_search_now,
v_ran_now: what a re-cut after a collision would use) while the integration
keeps the fixed ones; `recompute_cutoffs` applies new radii every step
instead.

overlap=True runs (4)-(7) as one p3t_hard_evaluate call: clusters still
running after 2^slow_log2 block steps park and finish on a second stream
while the tree of everyone else is evaluated, and their soft terms are
summed directly afterwards.  With
recompute_cutoffs the evaluation of step k then uses the radii computed from
the state of evaluation k-1 (the hard part of step k still uses the radii of
evaluation k-1, as the P3T split requires): the radii lag one step, because
the slow members' new state is not known when the tree is built.

collisions=(f, density) (serial path only) looks for perfect-accretion
collisions in the hard part (p3t_hard_step_collide, Section 2.5.1); after a
hard part with mergers the composites become single particles
(p3t_merge_bodies), the particle count drops, and the cut-off and search
radii of all particles are recomputed (step (9)) before the evaluation of
step (7), which then serves both the second kick and the next step.
`n_collisions` and `eps` (six sums, see p3t_hard_step_collide) accumulate
over the run.
"""
from __future__ import annotations

import torch

from .api import Context, Params


class P3TStepper:
    """graph=True evaluates tree + force through p3t_evaluate's captured
    hipGraph (replayed every step: positions, masses, radii and the
    acceleration live in fixed buffers)."""

    def __init__(self, ctx: Context, pos, vel, mass, recompute_cutoffs: bool = False, graph: bool = False,
                 fused_hard: bool = True, overlap: bool = False, slow_log2: int = 9, monitor_cutoffs: bool = False,
                 collisions: tuple[float, float] | None = None):
        if collisions is not None and (graph or overlap or not fused_hard):
            raise ValueError("collisions run on the serial path (graph=False, overlap=False, fused_hard=True)")
        self.ctx = ctx
        self.collisions = collisions
        self.n_collisions = 0
        self.eps = [0.0] * 6
        self.merged = torch.empty(int(mass.shape[0]), dtype=torch.int32, device=pos.device)
        self.graph = graph
        self.fused_hard = fused_hard
        self.overlap = overlap
        self.slow_log2 = slow_log2
        self.n_slow = 0
        self.pos, self.vel, self.mass = pos, vel, mass
        self.n = int(mass.shape[0])
        self.dt = ctx.params.dt_soft
        self.recompute = recompute_cutoffs
        self.r_out, self.r_search, self.v_ran = ctx.compute_cutoffs(pos, vel, mass)
        self.monitor = monitor_cutoffs and not recompute_cutoffs
        if self.monitor:
            self.r_out_now, self.r_search_now, self.v_ran_now = (t.clone() for t in (self.r_out, self.r_search,
                                                                                      self.v_ran))
        self.dt_hard = torch.zeros(self.n, dtype=torch.float64, device=pos.device)
        self.steps = torch.zeros(self.n, dtype=torch.int32, device=pos.device)  # block steps of each cluster
        self.acc = torch.empty((3, self.n), dtype=torch.float64, device=pos.device)
        self.n_clusters = 0
        self._evaluate()
        # radii of the next evaluation (the same buffers unless they lag)
        self.r_out_next, self.r_search_next = self.r_out, self.r_search
        if overlap and recompute_cutoffs:
            self.r_out_next, self.r_search_next = self.r_out.clone(), self.r_search.clone()
            self.v_ran_next = self.v_ran.clone()

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
        """Counters of the last evaluation (host copies; no wait)."""
        return self.ctx.stats()

    def step(self):
        c = self.ctx
        c.kick(self.acc, self.vel, 0.5 * self.dt)
        if self.overlap:
            _, self.n_clusters, self.n_slow = c.hard_evaluate(
                self.pos, self.vel, self.mass, self.r_out, self.dt_hard, self.steps, self.r_out_next,
                self.r_search_next, out=self.acc, slow_log2=self.slow_log2, graph=self.graph)
            if self.recompute:
                # the radii just used become those of the next hard part;
                # the next evaluation's come from the state at hand.  A
                # captured evaluation keeps its buffers (copy); otherwise the
                # two sets simply trade places.
                if self.graph:
                    self.r_out.copy_(self.r_out_next)
                    self.r_search.copy_(self.r_search_next)
                    self.v_ran.copy_(self.v_ran_next)
                else:
                    self.r_out, self.r_out_next = self.r_out_next, self.r_out
                    self.r_search, self.r_search_next = self.r_search_next, self.r_search
                    self.v_ran, self.v_ran_next = self.v_ran_next, self.v_ran
                c.compute_cutoffs(self.pos, self.vel, self.mass,
                                  out=(self.r_out_next, self.r_search_next, self.v_ran_next))
            elif self.monitor:
                c.compute_cutoffs(self.pos, self.vel, self.mass, out=(self.r_out_now, self.r_search_now, self.v_ran_now))
            c.kick(self.acc, self.vel, 0.5 * self.dt)
            return
        if self.collisions is not None:
            f, rho = self.collisions
            self.n_clusters, nco, eps = c.hard_step_collide(self.pos, self.vel, self.mass, self.r_out, self.merged, f,
                                                            rho, dt_hard=self.dt_hard, steps=self.steps)
            self.n_collisions += nco
            self.eps = [a + b for a, b in zip(self.eps, eps)]
            if nco > 0:
                self._merge()
                self.r_out, self.r_search, self.v_ran = c.compute_cutoffs(self.pos, self.vel, self.mass)
        elif self.fused_hard:
            self.n_clusters = c.hard_step(self.pos, self.vel, self.mass, self.r_out, dt_hard=self.dt_hard,
                                          steps=self.steps)
        else:
            cl_ptr, members = c.clusters(self.label)
            self.n_clusters = int(cl_ptr.shape[0]) - 1
            c.hermite_cluster_step(self.pos, self.vel, self.mass, self.r_out, cl_ptr, members, dt_hard=self.dt_hard,
                                   energy=False)
        if self.recompute:
            c.compute_cutoffs(self.pos, self.vel, self.mass, out=(self.r_out, self.r_search, self.v_ran))
        elif self.monitor:
            c.compute_cutoffs(self.pos, self.vel, self.mass, out=(self.r_out_now, self.r_search_now, self.v_ran_now))
        self._evaluate()
        c.kick(self.acc, self.vel, 0.5 * self.dt)

    def _merge(self):
        """Composites to single particles, arrays compacted in place; the
        tensors become views of their first entries."""
        nn = self.ctx.merge_bodies(self.merged, self.pos, self.vel, self.mass, dt_hard=self.dt_hard, steps=self.steps)
        self.pos = self.pos.view(-1)[:3 * nn].view(3, nn)
        self.vel = self.vel.view(-1)[:3 * nn].view(3, nn)
        self.mass = self.mass[:nn]
        self.dt_hard = self.dt_hard[:nn]
        self.steps = self.steps[:nn]
        self.merged = self.merged[:nn]
        self.acc = torch.empty((3, nn), dtype=torch.float64, device=self.pos.device)
        self.n = nn

    def interactions(self) -> int:
        s = self.last
        return int(s["n_near"] + s["n_far"] + s["n_cell"])


__all__ = ["P3TStepper", "Params"]
