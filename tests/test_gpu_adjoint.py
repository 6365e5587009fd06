"""GPU parity of the soft-kick adjoint and the differentiable leapfrog.

* The frozen-list force equals the force of the same tree bit for bit.
* theta = 0 (every interaction a particle pair): the adjoint equals the
  oracle's direct vector-Jacobian product to 1e-12 of its largest entry.
* theta = 0.5 with monopole cells: the adjoint equals central finite
  differences of the frozen-list force (the function it differentiates) to
  1e-6 of the largest entry (FP64 differences of relative size 1e-7).
* Leapfrog with checkpointing: the autograd gradient of sum |x_final|^2 with
  respect to the initial positions and the masses equals the oracle leapfrog
  adjoint (theta = 0) to 1e-9, and checkpointing changes it by no more than
  the rounding of the adjoint's atomic sums.
"""
import numpy as np
import pytest
import torch

import diskgen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def setup(gpu, orc, disk, **kw):
    p = orc.Params()
    ro, rs, _ = orc.cutoffs(disk.pos, disk.vel, disk.mass, p)
    ctx = gpu.Context(gpu.Params.defaults().replace(**kw))
    g = dict(pos=T(disk.pos), vel=T(disk.vel), m=T(disk.mass), ro=T(ro), rs=T(rs))
    ctx.build_tree(g["pos"], g["vel"], g["m"], g["ro"], g["rs"])
    acc = ctx.compute_soft_force()
    return ctx, g, acc, ro, p


@pytest.mark.parametrize("multipole", [1, 2])
def test_frozen_force_equals_force(gpu, orc, multipole):
    d = diskgen.workload("disk2k_equal")
    ctx, g, acc, _, _ = setup(gpu, orc, d, theta=0.5, multipole=multipole)
    acc2 = ctx.soft_force_frozen(g["pos"], g["m"])
    assert torch.equal(acc, acc2)


def test_adjoint_theta0_matches_oracle(gpu, orc):
    d = diskgen.workload("disk2k_equal")
    ctx, g, acc, ro, p = setup(gpu, orc, d, theta=0.0, multipole=2)
    lam = np.random.default_rng(5).normal(size=(3, d.n))
    gx, gm = ctx.soft_kick_adjoint(T(lam), 0.5)
    ogx, ogm = orc.soft_adjoint(d.pos, d.mass, ro, lam, p)
    ex = np.abs(gx.cpu().numpy() - 0.5 * ogx).max() / np.abs(0.5 * ogx).max()
    em = np.abs(gm.cpu().numpy() - 0.5 * ogm).max() / np.abs(0.5 * ogm).max()
    print("adjoint vs oracle (theta=0): x", ex, "m", em)
    assert ex < 1e-12 and em < 1e-12


def fd_check(ctx, g, n, lam, idx, gx, gm, dx):
    """Central differences of L = lam . a_frozen at the particles idx."""
    pos, m = g["pos"], g["m"]
    worst_x = worst_m = 0.0
    sx, sm = gx.abs().max().item(), gm.abs().max().item()
    for k in idx:
        for c in range(3):
            pp = pos.clone()
            pp[c, k] += dx
            ap = ctx.soft_force_frozen(pp, m)
            pp[c, k] -= 2 * dx
            am = ctx.soft_force_frozen(pp, m)
            fd = (lam * (ap - am)).sum().item() / (2 * dx)
            worst_x = max(worst_x, abs(fd - gx[c, k].item()) / sx)
        dm = 1e-6 * m[k].item()
        mp = m.clone()
        mp[k] += dm
        ap = ctx.soft_force_frozen(pos, mp)
        mp[k] -= 2 * dm
        am = ctx.soft_force_frozen(pos, mp)
        fd = (lam * (ap - am)).sum().item() / (2 * dm)
        worst_m = max(worst_m, abs(fd - gm[k].item()) / sm)
    return worst_x, worst_m


@pytest.mark.parametrize("workload,n,n_fd", [("disk2k_equal", None, 24), ("disk256k_masslaw", None, 64)])
def test_adjoint_matches_finite_differences(gpu, orc, workload, n, n_fd):
    """theta = 0.5 monopole; the 2^18-particle disk is the differentiable
    configuration's size (64 sampled particles)."""
    d = diskgen.workload(workload, n)
    ctx, g, acc, _, _ = setup(gpu, orc, d, theta=0.5, multipole=1)
    assert ctx.stats()["n_cell"] > 0
    lam = T(np.random.default_rng(6).normal(size=(3, d.n)))
    gx, gm = ctx.soft_kick_adjoint(lam, 1.0)
    idx = diskgen.sample_indices(d.n, n_fd, 55)
    wx, wm = fd_check(ctx, g, d.n, lam, idx, gx, gm, 1e-9)
    print(workload, "adjoint vs central differences: x", wx, "m", wm)
    assert wx < 1e-6 and wm < 1e-6


def test_adjoint_rejects_quadrupole_cells(gpu, orc):
    d = diskgen.workload("disk2k_equal")
    ctx, g, acc, _, _ = setup(gpu, orc, d, theta=0.5, multipole=2)
    with pytest.raises(gpu.P3TError):
        ctx.soft_kick_adjoint(T(np.ones((3, d.n))), 1.0)


@pytest.mark.parametrize("n,steps,every", [(1024, 4, 2), (16384, 16, 4)])
def test_leapfrog_gradient_matches_oracle(gpu, orc, n, steps, every):
    from oracle import leapfrog as olf
    from paper_2007_15432_amd.autodiff import leapfrog

    d = diskgen.workload("disk256k_masslaw", n)
    p = orc.Params()
    ro, rs, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
    ctx = gpu.Context(gpu.Params.defaults().replace(theta=0.0, multipole=1))
    h = p.dt_soft
    grads = []
    for ck in (every, 0) if n <= 1024 else (every,):
        x = T(d.pos).requires_grad_(True)
        m = T(d.mass).requires_grad_(True)
        xf, vf = leapfrog(x, T(d.vel), m, T(ro), T(rs), ctx, h, steps, checkpoint_every=ck)
        (xf * xf).sum().backward()
        grads.append((x.grad.cpu().numpy(), m.grad.cpu().numpy()))
    if len(grads) == 2:
        # recomputation gives the same forward; the adjoint's atomic sums may
        # round differently from run to run
        for a, b in zip(grads[0], grads[1]):
            assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    xo, vo, tape = olf.leapfrog(d.pos, d.vel, d.mass, ro, p, h, steps)
    lx, lv, lm = olf.leapfrog_adjoint(d.mass, ro, p, h, tape, 2.0 * xo, np.zeros_like(vo))
    gx, gm = grads[0]
    ex = np.abs(gx - lx).max() / np.abs(lx).max()
    em = np.abs(gm - lm).max() / np.abs(lm).max()
    print(f"leapfrog n={n} steps={steps}: x {ex:.3e} m {em:.3e}")
    assert ex < 1e-9 and em < 1e-9


def test_leapfrog_full_size_checkpointed(gpu, orc):
    """The differentiable configuration at full size: 2^18 particles, 16
    kick-drift-kick steps, theta = 0.5 monopole cells, checkpoint every 4
    steps.  The checkpointed gradient equals the stored-tape gradient up to
    the rounding of the adjoint's atomic sums (the recomputed forward is the
    same to the bit), and every entry is finite."""
    import time

    from paper_2007_15432_amd.autodiff import leapfrog

    d = diskgen.workload("disk256k_masslaw")
    p = orc.Params()
    ro, rs, _ = orc.cutoffs(d.pos, d.vel, d.mass, p)
    ctx = gpu.Context(gpu.Params.defaults().replace(theta=0.5, multipole=1))
    ctx.reserve(d.n, 4 * d.n)
    out = []
    for ck in (4, 0):
        x = T(d.pos).requires_grad_(True)
        m = T(d.mass).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xf, vf = leapfrog(x, T(d.vel), m, T(ro), T(rs), ctx, p.dt_soft, 16, checkpoint_every=ck)
        (xf * xf).sum().backward()
        torch.cuda.synchronize()
        print(f"n={d.n} 16 steps checkpoint_every={ck}: forward+backward {time.perf_counter() - t0:.2f} s")
        out.append((x.grad.clone(), m.grad.clone()))
    for a, b in zip(out[0], out[1]):
        assert torch.isfinite(a).all()
        assert (a - b).abs().max().item() <= 1e-10 * b.abs().max().item()


def test_adjoint_mixed_precision(gpu, orc):
    """precision = 1: the K = 1 terms of the adjoint in FP32 (as in the
    forward force).  Against the FP64 adjoint of the same tree and lists:
    within 1e-5 of the largest entry (FP32 rounding of each term, summed in
    FP64); against central differences of the FP64 frozen force at 64
    sampled particles of the 2^18-particle disk: within 1e-3."""
    import time

    d = diskgen.workload("disk256k_masslaw")
    ctx64, g, _, _, _ = setup(gpu, orc, d, theta=0.5, multipole=1)
    ctx32, _, _, _, _ = setup(gpu, orc, d, theta=0.5, multipole=1, precision=1)
    lam = T(np.random.default_rng(6).normal(size=(3, d.n)))
    out = {}
    for name, ctx in (("fp64", ctx64), ("mixed", ctx32)):
        ctx.soft_kick_adjoint(lam, 1.0)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            gx, gm = ctx.soft_kick_adjoint(lam, 1.0)
        torch.cuda.synchronize()
        out[name] = (gx, gm, 1e3 * (time.perf_counter() - t0) / 5)
    gx64, gm64, t64 = out["fp64"]
    gx32, gm32, t32 = out["mixed"]
    ex = ((gx32 - gx64).abs().max() / gx64.abs().max()).item()
    em = ((gm32 - gm64).abs().max() / gm64.abs().max()).item()
    print(f"adjoint ms: fp64 {t64:.3f}, mixed {t32:.3f}; mixed vs fp64: x {ex:.2e}, m {em:.2e}")
    assert ex < 1e-5 and em < 1e-5
    idx = diskgen.sample_indices(d.n, 64, 55)
    wx, wm = fd_check(ctx64, g, d.n, lam, idx, gx32, gm32, 1e-9)
    print("mixed adjoint vs central differences of the FP64 force: x", wx, "m", wm)
    assert wx < 1e-3 and wm < 1e-3
