"""Thin Python binding of libp3t: argument marshalling for torch tensors.

Every computation runs in the library's HIP kernels; this module only checks
tensor shapes / dtypes / devices and passes device pointers and the current
HIP stream through the C ABI.  Particle arrays are (3, n) float64 (rows x, y,
z) or (n,) float64, on the context's GPU, contiguous.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, fields

import torch

from . import _lib

__all__ = ["Params", "Context", "P3TError", "compute_cutoffs_noalloc"]


class P3TError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


@dataclass
class Params:
    """Mirror of p3t_params (include/p3t.h); defaults from p3t_default_params."""

    G: float = 1.0
    m_star: float = 1.0
    gamma: float = 0.1
    r_cut0: float = 2.0
    r_cut1: float = 8.0
    r_search0: float = 1.1
    r_search1: float = 6.0
    r_search2: float = 2.0
    r_search3: float = 2.0
    dt_soft: float = 0.09817477042468103
    theta: float = 0.5
    eta: float = 0.01
    eta0: float = 0.001
    multipole: int = 2
    precision: int = 0
    cutoff_mode: int = 0
    hill_length: int = 0
    n_group_max: int = 128
    n_leaf_max: int = 16
    vran_bins: int = 64
    vran_min_count: int = 8
    k_max: int = 40
    cluster_cap: int = 1024
    isolated: int = 0

    @classmethod
    def defaults(cls) -> "Params":
        cp = _lib.CParams()
        _lib.load().p3t_default_params(C.byref(cp))
        return cls(**{f.name: getattr(cp, f.name) for f in fields(cls)})

    def to_c(self) -> _lib.CParams:
        return _lib.CParams(**{f.name: getattr(self, f.name) for f in fields(self)})

    def replace(self, **kw) -> "Params":
        d = {f.name: getattr(self, f.name) for f in fields(self)}
        d.update(kw)
        return Params(**d)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """One library context bound to a GPU; owns the library's scratch."""

    def __init__(self, params: Params | None = None, device: int | str | torch.device = 0):
        self.L = _lib.load()
        idx = device if isinstance(device, int) else (torch.device(device).index or 0)
        self.device = torch.device("cuda", idx)
        self.params = params if params is not None else Params.defaults()
        self.n = 0
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = self.L.p3t_create(C.byref(self.params.to_c()), C.c_void_p(self._stream()), C.byref(self._h))
        if st != 0:
            raise P3TError(st, "p3t_create failed (invalid parameters or no device)")

    # -- plumbing ------------------------------------------------------------
    def _stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def _bind(self):
        self.L.p3t_set_stream(self._h, C.c_void_p(self._stream()))

    def _check(self, st: int, what: str):
        if st != 0:
            msg = self.L.p3t_last_error(self._h)
            raise P3TError(st, f"{what}: {msg.decode() if msg else ''}")

    def _vec3(self, t, n, name):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.device == self.device
                and tuple(t.shape) == (3, n) and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 (3, {n}) tensor on {self.device}")
        return t

    def _vec(self, t, n, name, dtype=torch.float64):
        if not (isinstance(t, torch.Tensor) and t.dtype == dtype and t.device == self.device
                and tuple(t.shape) == (n,) and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dtype} ({n},) tensor on {self.device}")
        return t

    def close(self):
        if self._h:
            self.L.p3t_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        self._check(self.L.p3t_set_params(self._h, C.byref(params.to_c())), "set_params")
        self.params = params

    def reserve(self, n_max: int, nnz_max: int = 0):
        self._check(self.L.p3t_reserve(self._h, int(n_max), int(nnz_max)), "reserve")

    def set_timing(self, on: bool = True):
        self._check(self.L.p3t_set_timing(self._h, 1 if on else 0), "set_timing")

    KERNEL_KEYS = ("force_split", "force_unroll", "force_persistent", "waves_per_cu", "walk_waves_per_cu",
                   "direct_pair_cap", "top_slots")

    def kernel_config(self) -> dict:
        k = _lib.CKernelConfig()
        self._check(self.L.p3t_get_kernel_config(self._h, C.byref(k)), "get_kernel_config")
        return {f: getattr(k, f) for f in self.KERNEL_KEYS}

    def set_kernel_config(self, **kw) -> dict:
        """Change launch shapes (see p3t_kernel_config); returns the new shape."""
        cur = self.kernel_config()
        bad = set(kw) - set(self.KERNEL_KEYS)
        if bad:
            raise ValueError(f"unknown kernel config keys {sorted(bad)}")
        cur.update(kw)
        k = _lib.CKernelConfig(*(int(cur[f]) for f in self.KERNEL_KEYS))
        self._check(self.L.p3t_set_kernel_config(self._h, C.byref(k)), "set_kernel_config")
        return cur

    def stats(self) -> dict:
        s = _lib.CStats()
        self._check(self.L.p3t_get_stats(self._h, C.byref(s)), "get_stats")
        return {f[0]: getattr(s, f[0]) for f in _lib.CStats._fields_}

    def status(self) -> int:
        v = C.c_uint32()
        self._check(self.L.p3t_get_status(self._h, C.byref(v)), "get_status")
        return int(v.value)

    # -- the hot path --------------------------------------------------------
    def compute_cutoffs(self, pos, vel, mass, out=None):
        """(r_out, r_search, v_ran), each (n,); out = (r_out, r_search, v_ran)
        tensors to write into (kept buffers keep a captured graph valid)."""
        n = int(mass.shape[0])
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        self._vec(mass, n, "mass")
        if out is not None:
            ro, rs, vr = out
            for t, name in ((ro, "r_out"), (rs, "r_search"), (vr, "v_ran")):
                self._vec(t, n, name)
        else:
            ro = torch.empty(n, dtype=torch.float64, device=self.device)
            rs = torch.empty_like(ro)
            vr = torch.empty_like(ro)
        self._bind()
        self._check(self.L.p3t_compute_cutoffs(self._h, n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(ro), _ptr(rs),
                                               _ptr(vr)), "compute_cutoffs")
        return ro, rs, vr

    def build_tree(self, pos, vel, mass, r_out, r_search):
        n = int(mass.shape[0])
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        for t, name in ((mass, "mass"), (r_out, "r_out"), (r_search, "r_search")):
            self._vec(t, n, name)
        self._bind()
        self._check(self.L.p3t_build_tree(self._h, n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(r_out), _ptr(r_search)),
                    "build_tree")
        self.n = n

    def compute_soft_force(self, out=None):
        n = self.n
        acc = out if out is not None else torch.empty((3, n), dtype=torch.float64, device=self.device)
        self._vec3(acc, n, "acc")
        self._bind()
        self._check(self.L.p3t_compute_soft_force(self._h, _ptr(acc)), "compute_soft_force")
        return acc

    def evaluate(self, pos, vel, mass, r_out, r_search, out=None, graph: bool = True):
        """build_tree + compute_soft_force; with graph=True the device sequence
        is captured once into a hipGraph and replayed."""
        n = int(mass.shape[0])
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        for t, name in ((mass, "mass"), (r_out, "r_out"), (r_search, "r_search")):
            self._vec(t, n, name)
        acc = out if out is not None else torch.empty((3, n), dtype=torch.float64, device=self.device)
        self._vec3(acc, n, "acc")
        self._bind()
        self._check(self.L.p3t_evaluate(self._h, n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(r_out), _ptr(r_search),
                                        _ptr(acc), 1 if graph else 0), "evaluate")
        self.n = n
        return acc

    def hard_step(self, pos, vel, mass, r_out, dt_hard=None, steps=None) -> int:
        """Clusters from the last evaluation's neighbour pairs and their
        Hermite integration over dt_soft, in place; returns the cluster count.
        `steps` (int32 (n,), nullable) receives each particle's cluster step
        count."""
        n = self.n
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        self._vec(mass, n, "mass")
        self._vec(r_out, n, "r_out")
        if dt_hard is not None:
            self._vec(dt_hard, n, "dt_hard")
        if steps is not None:
            self._vec(steps, n, "steps", dtype=torch.int32)
        nc = C.c_int64(0)
        self._bind()
        self._check(self.L.p3t_hard_step(self._h, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(r_out), _ptr(dt_hard),
                                         _ptr(steps), C.byref(nc)), "hard_step")
        return int(nc.value)

    def hard_step_collide(self, pos, vel, mass, r_out, merged_into, f_radius: float, density: float, dt_hard=None,
                          steps=None):
        """hard_step with perfect-accretion collisions (Section 2.5.1):
        merged_into (int32 (n,)) receives each particle's composite (lowest
        index).  Returns (clusters, mergers, eps (6 floats: eps_0..eps_3 with
        W, their total with W = 1, with 1 - W))."""
        n = self.n
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        self._vec(mass, n, "mass")
        self._vec(r_out, n, "r_out")
        self._vec(merged_into, n, "merged_into", dtype=torch.int32)
        if dt_hard is not None:
            self._vec(dt_hard, n, "dt_hard")
        if steps is not None:
            self._vec(steps, n, "steps", dtype=torch.int32)
        nc, ncoll = C.c_int64(0), C.c_int64(0)
        eps = (C.c_double * 6)()
        self._bind()
        self._check(self.L.p3t_hard_step_collide(self._h, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(r_out),
                                                 _ptr(dt_hard), _ptr(steps), float(f_radius), float(density),
                                                 _ptr(merged_into), eps, C.byref(ncoll), C.byref(nc)),
                    "hard_step_collide")
        return int(nc.value), int(ncoll.value), [float(x) for x in eps]

    def hermite_collide(self, pos, vel, mass, r_out, cl_ptr, members, f_radius: float, density: float, dt_hard=None,
                        energy: bool = True, steps: bool = False):
        """p3t_hermite_collide on caller-given clusters.  Returns a dict:
        merged_into (int32 (n,)), eps (float64 (nc, 6)), ncoll, and e_rel /
        nsteps when asked for."""
        n = int(mass.shape[0])
        nc = int(cl_ptr.shape[0]) - 1
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        self._vec(mass, n, "mass")
        self._vec(r_out, n, "r_out")
        if dt_hard is not None:
            self._vec(dt_hard, n, "dt_hard")
        dev = self.device
        merged = torch.empty(n, dtype=torch.int32, device=dev)
        eps = torch.empty((max(nc, 0), 6), dtype=torch.float64, device=dev)
        e_rel = torch.empty(max(nc, 0), dtype=torch.float64, device=dev) if energy else None
        ns = torch.empty(max(nc, 0), dtype=torch.int32, device=dev) if steps else None
        nco = C.c_int64(0)
        self._bind()
        self._check(self.L.p3t_hermite_collide(self._h, n, nc, _ptr(cl_ptr), _ptr(members), _ptr(pos), _ptr(vel),
                                               _ptr(mass), _ptr(r_out), _ptr(dt_hard), float(f_radius),
                                               float(density), _ptr(merged), _ptr(eps), _ptr(e_rel), _ptr(ns),
                                               C.byref(nco)), "hermite_collide")
        out = dict(merged_into=merged, eps=eps, ncoll=int(nco.value))
        if energy:
            out["e_rel"] = e_rel
        if steps:
            out["nsteps"] = ns
        return out

    def merge_bodies(self, merged_into, pos, vel, mass, dt_hard=None, steps=None) -> int:
        """Each composite becomes one particle (Section 2.5.1); the arrays are
        compacted in place (the first 3 n_new / n_new entries, row stride
        n_new).  Returns n_new; see merged_views for the compacted tensors."""
        n = int(mass.shape[0])
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        self._vec(mass, n, "mass")
        self._vec(merged_into, n, "merged_into", dtype=torch.int32)
        if dt_hard is not None:
            self._vec(dt_hard, n, "dt_hard")
        if steps is not None:
            self._vec(steps, n, "steps", dtype=torch.int32)
        nn = C.c_int64(0)
        self._bind()
        self._check(self.L.p3t_merge_bodies(self._h, n, _ptr(merged_into), _ptr(pos), _ptr(vel), _ptr(mass),
                                            _ptr(dt_hard), _ptr(steps), C.byref(nn)), "merge_bodies")
        return int(nn.value)

    def hard_evaluate(self, pos, vel, mass, r_out_hard, dt_hard, steps, r_out, r_search, out=None,
                      slow_log2: int = 9, graph: bool = True):
        """hard_step then evaluate in one call.  Clusters still running after
        2^slow_log2 block steps park and finish on a second stream while the
        tree of the others is evaluated; their soft terms are then summed
        directly.  `steps` (int32, nullable) receives each particle's cluster
        step count.  Returns (acc (3, n), clusters, parked members)."""
        n = self.n
        for a, nm in ((pos, "pos"), (vel, "vel")):
            self._vec3(a, n, nm)
        for a, nm in ((mass, "mass"), (r_out_hard, "r_out_hard"), (r_out, "r_out"), (r_search, "r_search")):
            self._vec(a, n, nm)
        if dt_hard is not None:
            self._vec(dt_hard, n, "dt_hard")
        if steps is not None:
            self._vec(steps, n, "steps", dtype=torch.int32)
        acc = out if out is not None else torch.empty((3, n), dtype=torch.float64, device=self.device)
        self._vec3(acc, n, "acc")
        nc, ns = C.c_int64(0), C.c_int64(0)
        self._bind()
        self._check(self.L.p3t_hard_evaluate(self._h, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(r_out_hard),
                                             _ptr(dt_hard), _ptr(steps), _ptr(r_out), _ptr(r_search), _ptr(acc),
                                             int(slow_log2), 1 if graph else 0, C.byref(nc), C.byref(ns)),
                    "hard_evaluate")
        return acc, int(nc.value), int(ns.value)

    def total_energy(self, pos, vel, mass) -> float:
        """Newtonian total energy of the particles about the star (eq. (soft)
        + eq. (hard)), direct O(N^2) with compensated sums."""
        n = int(mass.shape[0])
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        self._vec(mass, n, "mass")
        e = C.c_double(0.0)
        self._bind()
        self._check(self.L.p3t_total_energy(self._h, n, _ptr(pos), _ptr(vel), _ptr(mass), C.byref(e)), "total_energy")
        return float(e.value)

    def soft_force_frozen(self, pos, mass, out=None):
        """Soft force at new positions / masses over the current tree topology
        and interaction lists (the function the adjoint differentiates)."""
        n = self.n
        self._vec3(pos, n, "pos")
        self._vec(mass, n, "mass")
        acc = out if out is not None else torch.empty((3, n), dtype=torch.float64, device=self.device)
        self._vec3(acc, n, "acc")
        self._bind()
        self._check(self.L.p3t_soft_force_frozen(self._h, _ptr(pos), _ptr(mass), _ptr(acc)), "soft_force_frozen")
        return acc

    def soft_kick_adjoint(self, lam_v, h: float):
        """(h dL/dx (3, n), h dL/dm (n,)) for L = lam_v . a at the last force
        evaluation, lists and pair cut-offs held fixed."""
        n = self.n
        self._vec3(lam_v, n, "lam_v")
        gx = torch.empty((3, n), dtype=torch.float64, device=self.device)
        gm = torch.empty(n, dtype=torch.float64, device=self.device)
        self._bind()
        self._check(self.L.p3t_soft_kick_adjoint(self._h, float(h), _ptr(lam_v), _ptr(gx), _ptr(gm)),
                    "soft_kick_adjoint")
        return gx, gm

    def neighbour_list(self, labels: bool = True):
        """(row_ptr int64 (n+1,), col int32 (nnz,), label int32 (n,) or None)."""
        n = self.n
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        label = torch.empty(n, dtype=torch.int32, device=self.device) if labels else None
        nnz = C.c_int64(0)
        cap = max(1, getattr(self, "_nnz_hint", 1024))
        for _ in range(2):
            col = torch.empty(cap, dtype=torch.int32, device=self.device)
            self._bind()
            st = self.L.p3t_neighbour_list(self._h, _ptr(row_ptr), _ptr(col), cap, C.byref(nnz), _ptr(label))
            if st == _lib.P3T_ERR_CAPACITY:
                cap = int(nnz.value)
                self._nnz_hint = cap
                continue
            self._check(st, "neighbour_list")
            return row_ptr, col[: nnz.value], label
        raise P3TError(_lib.P3T_ERR_CAPACITY, "neighbour_list: capacity retry failed")

    def clusters(self, label):
        n = int(label.shape[0])
        self._vec(label, n, "label", torch.int32)
        cl_ptr = torch.empty(n + 1, dtype=torch.int32, device=self.device)
        members = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        nc = C.c_int64(0)
        self._bind()
        self._check(self.L.p3t_clusters(self._h, n, _ptr(label), _ptr(cl_ptr), _ptr(members), C.byref(nc)),
                    "clusters")
        return cl_ptr[: nc.value + 1], members[:n]

    def hermite_cluster_step(self, pos, vel, mass, r_out, cl_ptr, members, dt_hard=None, energy=True,
                             steps=False):
        """Integrate every cluster over one soft step in place; returns the
        per-cluster relative energy error (or None), and with steps=True also
        the per-cluster block-step counts."""
        n = int(mass.shape[0])
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        self._vec(mass, n, "mass")
        self._vec(r_out, n, "r_out")
        nc = int(cl_ptr.shape[0]) - 1
        self._vec(cl_ptr, nc + 1, "cl_ptr", torch.int32)
        self._vec(members, int(members.shape[0]), "members", torch.int32)
        if dt_hard is not None:
            self._vec(dt_hard, n, "dt_hard")
        err = torch.empty(max(nc, 1), dtype=torch.float64, device=self.device) if energy else None
        nst = torch.empty(max(nc, 1), dtype=torch.int32, device=self.device) if steps else None
        self._bind()
        self._check(self.L.p3t_hermite_cluster_step(self._h, n, nc, _ptr(cl_ptr), _ptr(members), _ptr(pos), _ptr(vel),
                                                    _ptr(mass), _ptr(r_out), _ptr(dt_hard), _ptr(err), _ptr(nst)),
                    "hermite_cluster_step")
        e = None if err is None else err[:nc]
        return (e, nst[:nc]) if steps else e

    def kick(self, acc, vel, h: float):
        n = int(vel.shape[1])
        self._vec3(acc, n, "acc")
        self._vec3(vel, n, "vel")
        self._bind()
        self._check(self.L.p3t_kick(self._h, n, float(h), _ptr(acc), _ptr(vel)), "kick")

    def kepler_drift(self, pos, vel, dt: float | None = None, index=None, iters: bool = False, count: bool = True):
        """Drift the listed particles (index: int32 tensor, None = all) for dt
        (default dt_soft) on their two-body orbits about the star, in place.
        Returns (n_unbound or None, per-entry Newton iterations or None)."""
        n = int(pos.shape[1])
        self._vec3(pos, n, "pos")
        self._vec3(vel, n, "vel")
        m = n
        if index is not None:
            m = int(index.shape[0])
            self._vec(index, m, "index", torch.int32)
        it = torch.empty(max(m, 1), dtype=torch.int32, device=self.device) if iters else None
        nu = C.c_int64(0)
        self._bind()
        self._check(self.L.p3t_kepler_drift(self._h, n, float(self.params.dt_soft if dt is None else dt), _ptr(pos),
                                            _ptr(vel), _ptr(index), m, _ptr(it),
                                            C.byref(nu) if count else None), "kepler_drift")
        return (int(nu.value) if count else None), (None if it is None else it[:m])


def compute_cutoffs_noalloc(params: Params, pos, vel, mass, out):
    """p3t_compute_cutoffs_noalloc: the cut-off and search radii without a
    context and without allocating, into out = (r_out, r_search, v_ran or
    None), on the current stream of the tensors' device."""
    L = _lib.load()
    n = int(mass.shape[0])
    dev = mass.device
    for t, shape, name in ((pos, (3, n), "pos"), (vel, (3, n), "vel"), (mass, (n,), "mass")):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.device == dev
                and tuple(t.shape) == shape and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 {shape} tensor on {dev}")
    ro, rs, vr = out
    for t, name in ((ro, "r_out"), (rs, "r_search"), (vr, "v_ran")):
        if t is None and name == "v_ran":
            continue
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.device == dev
                and tuple(t.shape) == (n,) and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 ({n},) tensor on {dev}")
    with torch.cuda.device(dev):
        st = L.p3t_compute_cutoffs_noalloc(C.byref(params.to_c()), n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(ro),
                                           _ptr(rs), _ptr(vr), C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    if st != 0:
        msg = L.p3t_last_error(None)
        raise P3TError(st, f"compute_cutoffs_noalloc: {msg.decode() if msg else ''}")
    return ro, rs, vr

