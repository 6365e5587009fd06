"""Autotuner for the tree / walk / force evaluation.

Picks the group and leaf sizes of the tree (which change the interaction
lists) and the launch shapes of the force and walk kernels (which change only
the order of floating-point summation) by timing the real evaluation on the
caller's particles with the library's event timers.  The objective is the
device time of one evaluation, tree + walk + force (p3t_stats ms_tree +
ms_walk + ms_force), median over repetitions.

The search is coordinate-wise, in three stages that each fix what the
previous stage chose:
  1. (n_group_max, n_leaf_max) with the default launch shapes;
  2. (force_split, force_unroll, waves_per_cu) on the chosen lists;
  3. walk_waves_per_cu.
Stage 1 respects an upper bound on the group size.  Every candidate is a
valid library configuration: the lists follow the same opening rule and the
neighbour lists are the same.  Group and leaf sizes do change which cells a
group accepts, hence the interaction count and the truncation error; a
caller that must keep the error fixed passes one group and one leaf size,
and then only the launch shapes, which change nothing but the order of
summation, are tuned.  With empty `shapes` and `walk_waves` only stage 1
runs (a sweep of list shapes).
"""
from __future__ import annotations

import itertools
import json
import statistics
import time
from dataclasses import asdict, dataclass, field

GROUPS = (64, 96, 128)
LEAVES = (8, 16, 32)
SHAPES = [dict(force_split=0, force_unroll=4)] + [
    dict(force_split=1, force_unroll=u, waves_per_cu=w) for u in (1, 2, 4, 8) for w in (8, 16, 32)]
WALK_WAVES = (2, 4, 8, 16)


@dataclass
class Trial:
    stage: int
    params: dict
    kernel: dict
    ms: float
    interactions: int


@dataclass
class TuneResult:
    params: dict
    kernel: dict
    ms: float
    trials: list = field(default_factory=list)
    seconds: float = 0.0
    sweep: list = field(default_factory=list)

    def to_json(self) -> str:
        return json.dumps({"params": self.params, "kernel": self.kernel, "ms": self.ms, "seconds": self.seconds,
                           "trials": [asdict(t) for t in self.trials]})


def _best(trials, incumbent=None, margin: float = 0.03):
    """Fastest trial; the incumbent stays unless beaten by more than
    `margin` (timing noise would otherwise flip between equal shapes)."""
    b = min(trials, key=lambda t: t.ms)
    if incumbent is not None and incumbent.ms <= b.ms * (1.0 + margin):
        return incumbent
    return b


def search(measure, group_cap: int = 128, groups=GROUPS, leaves=LEAVES, shapes=SHAPES, walk_waves=WALK_WAVES,
           default_kernel=None) -> TuneResult:
    """Coordinate search driven by measure(params: dict, kernel: dict) ->
    (ms, interactions).  Host logic only; see tune() for the GPU measure."""
    kernel0 = dict(default_kernel or dict(force_split=1, force_unroll=4, force_persistent=1, waves_per_cu=8,
                                          walk_waves_per_cu=8))
    trials = []
    s1 = []
    for g, l in itertools.product(groups, leaves):
        if g > group_cap or l > g:
            continue
        p = dict(n_group_max=g, n_leaf_max=l)
        ms, inter = measure(p, kernel0)
        s1.append(Trial(1, p, dict(kernel0), ms, inter))
    if not s1:
        raise ValueError("no group/leaf candidate within the group-size cap")
    b1 = _best(s1)
    if not shapes and not walk_waves:
        return TuneResult(params=dict(b1.params), kernel=dict(b1.kernel), ms=b1.ms, trials=s1)
    s2 = []
    for sh in shapes:
        k = dict(kernel0)
        k.update(sh)
        ms, inter = measure(b1.params, k)
        s2.append(Trial(2, dict(b1.params), k, ms, inter))
    b2 = _best(s2, incumbent=b1)
    s3 = []
    for w in walk_waves:
        k = dict(b2.kernel)
        k["walk_waves_per_cu"] = w
        ms, inter = measure(b2.params, k)
        s3.append(Trial(3, dict(b2.params), k, ms, inter))
    b3 = _best(s3, incumbent=b2)
    trials = s1 + s2 + s3
    return TuneResult(params=dict(b3.params), kernel=dict(b3.kernel), ms=b3.ms, trials=trials)


def tune(ctx, pos, vel, mass, r_out, r_search, reps: int = 3, group_cap: int = 128, **space) -> TuneResult:
    """Tune `ctx` on these particles (device tensors as for build_tree) and
    leave it configured with the winner.  Returns the full trial table."""
    base = ctx.params
    t0 = time.perf_counter()

    def measure(p, k):
        ctx.set_params(base.replace(**p))
        ctx.set_kernel_config(**k)
        ctx.set_timing(True)
        times = []
        inter = 0
        for r in range(reps + 1):
            ctx.build_tree(pos, vel, mass, r_out, r_search)
            ctx.compute_soft_force()
            s = ctx.stats()
            inter = int(s["n_near"] + s["n_far"] + s["n_cell"])
            if r > 0:  # the first run pays for buffer growth
                times.append(s["ms_tree"] + s["ms_walk"] + s["ms_force"])
        ctx.set_timing(False)
        return statistics.median(times), inter

    res = search(measure, group_cap=group_cap, **space)
    ctx.set_params(base.replace(**res.params))
    ctx.set_kernel_config(**res.kernel)
    res.seconds = time.perf_counter() - t0
    return res
