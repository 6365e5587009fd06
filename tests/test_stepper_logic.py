"""Host logic of the step driver (P3TStepper), on the CPU with a stand-in
context that records what the library calls receive.

With the overlapped hard part and recomputed cut-off radii, the radii lag one
step: the hard part of step k must use the radii of evaluation k-1 (the P3T
split pairs each soft evaluation with the hard part that follows it), and
evaluation k uses radii computed from the state of evaluation k-1.  A captured
evaluation must keep its radius buffers from step to step; an eager one may
trade them.
"""
import torch

from paper_2007_15432_amd.driver import P3TStepper


class _Params:
    dt_soft = 0.1


class FakeContext:
    """Radii carry a generation number: compute_cutoffs call g fills g."""

    def __init__(self):
        self.params = _Params()
        self.gen = 0
        self.calls = []

    def compute_cutoffs(self, pos, vel, mass, out=None):
        self.gen += 1
        n = int(mass.shape[0])
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float64) for _ in range(3))
        for t in out:
            t.fill_(float(self.gen))
        return out

    def build_tree(self, pos, vel, mass, r_out, r_search):
        self.calls.append(("tree", float(r_out[0]), r_out.data_ptr()))

    def compute_soft_force(self, out=None):
        return out

    def evaluate(self, pos, vel, mass, r_out, r_search, out=None, graph=True):
        self.calls.append(("evaluate", float(r_out[0]), r_out.data_ptr()))
        return out

    def kick(self, acc, vel, h):
        pass

    def hard_evaluate(self, pos, vel, mass, r_out_hard, dt_hard, steps, r_out, r_search, out=None, slow_log2=9,
                      graph=True):
        self.calls.append(("hard_evaluate", float(r_out_hard[0]), float(r_out[0]), float(r_search[0]),
                           r_out.data_ptr()))
        return out, 1, 0


def run(graph, steps=4):
    n = 8
    ctx = FakeContext()
    pos = torch.zeros((3, n), dtype=torch.float64)
    st = P3TStepper(ctx, pos, pos.clone(), torch.ones(n, dtype=torch.float64), recompute_cutoffs=True, graph=graph,
                    overlap=True)
    for _ in range(steps):
        st.step()
    return ctx, [c for c in ctx.calls if c[0] == "hard_evaluate"]


def test_overlapped_radii_lag_one_step():
    for graph in (False, True):
        ctx, he = run(graph)
        # initial radii: generation 1, used by the initial evaluation and by
        # the first step on both sides
        assert he[0][1:4] == (1.0, 1.0, 1.0)
        for k in range(1, len(he)):
            hard, ev, rs = he[k][1:4]
            assert hard == float(k), (graph, k, he[k])  # radii of the previous evaluation
            assert ev == rs == float(k + 1), (graph, k, he[k])  # computed after the previous step
        assert ctx.gen == len(he) + 1


def test_captured_evaluation_keeps_its_radius_buffer():
    _, he = run(graph=True)
    assert len({c[4] for c in he}) == 1
    _, he = run(graph=False)
    assert len({c[4] for c in he}) == 2  # eager: the two sets trade places


def test_serial_step_recomputes_before_the_evaluation():
    """Without the overlap the radii are recomputed after the hard part and
    before the tree, from the post-drift state (no lag)."""
    ctx = FakeContext()
    n = 4
    pos = torch.zeros((3, n), dtype=torch.float64)

    def hard_step(pos, vel, mass, r_out, dt_hard=None, steps=None):
        ctx.calls.append(("hard_step", float(r_out[0])))
        return 1

    ctx.hard_step = hard_step
    st = P3TStepper(ctx, pos, pos.clone(), torch.ones(n, dtype=torch.float64), recompute_cutoffs=True)
    st.step()
    st.step()
    seq = [c[:2] for c in ctx.calls]
    assert seq == [("tree", 1.0), ("hard_step", 1.0), ("tree", 2.0), ("hard_step", 2.0), ("tree", 3.0)]
