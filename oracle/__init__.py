"""CPU oracle for the P3T soft-force hot path (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use this package.  The GPU library never imports, links or calls
it, and this package never imports the GPU library.

The arithmetic lives in ``p3t_oracle.c`` (plain C, FP64, O(N^2)); this module
builds it with gcc on first use and exposes numpy-friendly wrappers.
Arrays of positions / velocities are (3, n) float64, C-contiguous.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "p3t_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# status bits returned by the oracle's C functions
ERR_COINCIDENT = 1
ERR_KMAX = 2
ERR_NSTEPS = 4
ERR_NAN = 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("G", C.c_double), ("m_star", C.c_double), ("gamma", C.c_double),
        ("r_cut0", C.c_double), ("r_cut1", C.c_double),
        ("r_search0", C.c_double), ("r_search1", C.c_double),
        ("r_search2", C.c_double), ("r_search3", C.c_double),
        ("dt_soft", C.c_double), ("eta", C.c_double), ("eta0", C.c_double),
        ("hill_length", C.c_int32), ("vran_bins", C.c_int32),
        ("vran_min_count", C.c_int32), ("k_max", C.c_int32), ("cutoff_mode", C.c_int32),
    ]


@dataclass
class Params:
    """Physical and method parameters (Section 3.1 of the paper; readings
    where it is silent: gamma = 0.1, Rcut0 = 2, dt = 2 pi / 64)."""

    G: float = 1.0
    m_star: float = 1.0
    gamma: float = 0.1
    r_cut0: float = 2.0
    r_cut1: float = 8.0
    r_search0: float = 1.1
    r_search1: float = 6.0
    r_search2: float = 2.0
    r_search3: float = 2.0
    dt_soft: float = 2.0 * np.pi / 64.0
    eta: float = 0.01
    eta0: float = 0.001
    hill_length: int = 0
    vran_bins: int = 64
    vran_min_count: int = 8
    k_max: int = 40
    cutoff_mode: int = 0  # 0: individual radii (eq. (rout2)), 1: shared (eq. (rout1))

    def c(self) -> _Params:
        return _Params(self.G, self.m_star, self.gamma, self.r_cut0, self.r_cut1,
                       self.r_search0, self.r_search1, self.r_search2, self.r_search3,
                       self.dt_soft, self.eta, self.eta0, self.hill_length,
                       self.vran_bins, self.vran_min_count, self.k_max, self.cutoff_mode)


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        dp, ip, i32p = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        pp = C.POINTER(_Params)
        for name in ("orc_W", "orc_dWdy", "orc_K", "orc_dKdy"):
            f = getattr(L, name)
            f.restype = C.c_double
            f.argtypes = [C.c_double, C.c_double]
        L.orc_cutoffs.argtypes = [C.c_int64, dp, dp, dp, pp, dp, dp, dp]
        L.orc_soft_acc.argtypes = [C.c_int64, dp, dp, dp, C.c_double, C.c_double, C.c_int64, ip, dp]
        L.orc_newton_acc.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_int64, ip, dp]
        L.orc_soft_energy.argtypes = [C.c_int64, dp, dp, dp, C.c_double, C.c_double]
        L.orc_soft_energy.restype = C.c_double
        L.orc_hard_acc_jerk.argtypes = [C.c_int64, dp, dp, dp, dp, pp, dp, dp]
        L.orc_cluster_energy.argtypes = [C.c_int64, dp, dp, dp, dp, pp]
        L.orc_cluster_energy.restype = C.c_double
        L.orc_hermite_one.argtypes = [C.c_int64, dp, dp, dp, dp, pp, C.c_double, dp, ip]
        L.orc_hermite_clusters.argtypes = [C.c_int64, C.c_int64, i32p, i32p, dp, dp, dp, dp, pp,
                                           C.c_double, dp, dp, dp, ip]
        L.orc_hermite_collide_clusters.argtypes = [C.c_int64, C.c_int64, i32p, i32p, dp, dp, dp, dp, pp,
                                                   C.c_double, dp, C.c_double, C.c_double, i32p, dp, dp, dp, ip,
                                                   ip, ip]
        L.orc_neighbour_rows.argtypes = [C.c_int64, dp, dp, dp, dp, dp, pp, C.c_int64, ip, ip, i32p,
                                         C.c_int64]
        L.orc_neighbour_rows.restype = C.c_int64
        L.orc_is_neighbour.argtypes = [dp, dp, pp]
        L.orc_labels.argtypes = [C.c_int64, ip, i32p, i32p]
        L.orc_soft_adjoint.argtypes = [C.c_int64, dp, dp, dp, C.c_double, C.c_double, dp, dp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _i32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> int:
    """Threads of later oracle calls; returns the count now in effect."""
    return int(lib().orc_set_threads(int(n)))


# -- changeover functions -------------------------------------------------
def W(y, gamma: float):
    f = lib().orc_W
    return np.vectorize(lambda t: f(float(t), gamma), otypes=[float])(y)


def dWdy(y, gamma: float):
    f = lib().orc_dWdy
    return np.vectorize(lambda t: f(float(t), gamma), otypes=[float])(y)


def K(y, gamma: float):
    f = lib().orc_K
    return np.vectorize(lambda t: f(float(t), gamma), otypes=[float])(y)


def dKdy(y, gamma: float):
    f = lib().orc_dKdy
    return np.vectorize(lambda t: f(float(t), gamma), otypes=[float])(y)


# -- cut-off radii ----------------------------------------------------------
def cutoffs(pos, vel, mass, p: Params):
    """(r_out, r_search, v_ran), each (n,)."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos, vel = _f64(pos, (3, n)), _f64(vel, (3, n))
    ro, rs, vr = np.empty(n), np.empty(n), np.empty(n)
    pc = p.c()
    lib().orc_cutoffs(n, _d(pos), _d(vel), _d(mass), C.byref(pc), _d(ro), _d(rs), _d(vr))
    return ro, rs, vr


# -- forces -------------------------------------------------------------------
def soft_acc(pos, mass, r_out, p: Params, idx=None):
    """Soft acceleration (3, ni) of particles idx (default all) from all."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos, r_out = _f64(pos, (3, n)), _f64(r_out, (n,))
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    acc = np.empty((3, idx.shape[0]))
    err = lib().orc_soft_acc(n, _d(pos), _d(mass), _d(r_out), p.G, p.gamma, idx.shape[0], _i64(idx), _d(acc))
    if err:
        raise FloatingPointError(f"oracle soft_acc status {err}")
    return acc


def newton_acc(pos, mass, G: float = 1.0, idx=None):
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n))
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    acc = np.empty((3, idx.shape[0]))
    lib().orc_newton_acc(n, _d(pos), _d(mass), G, idx.shape[0], _i64(idx), _d(acc))
    return acc


def soft_energy(pos, mass, r_out, p: Params) -> float:
    mass = _f64(mass)
    n = mass.shape[0]
    pos, r_out = _f64(pos, (3, n)), _f64(r_out, (n,))
    return float(lib().orc_soft_energy(n, _d(pos), _d(mass), _d(r_out), p.G, p.gamma))


def hard_acc_jerk(pos, vel, mass, r_out, p: Params):
    mass = _f64(mass)
    n = mass.shape[0]
    pos, vel, r_out = _f64(pos, (3, n)), _f64(vel, (3, n)), _f64(r_out, (n,))
    a, j = np.empty((3, n)), np.empty((3, n))
    pc = p.c()
    err = lib().orc_hard_acc_jerk(n, _d(pos), _d(vel), _d(mass), _d(r_out), C.byref(pc), _d(a), _d(j))
    if err:
        raise FloatingPointError(f"oracle hard_acc_jerk status {err}")
    return a, j


def cluster_energy(pos, vel, mass, r_out, p: Params) -> float:
    mass = _f64(mass)
    n = mass.shape[0]
    pos, vel, r_out = _f64(pos, (3, n)), _f64(vel, (3, n)), _f64(r_out, (n,))
    pc = p.c()
    return float(lib().orc_cluster_energy(n, _d(pos), _d(vel), _d(mass), _d(r_out), C.byref(pc)))


# -- Hermite ------------------------------------------------------------------
def hermite_clusters(pos, vel, mass, r_out, cl_ptr, members, p: Params, dt_soft=None, dt_hard=None):
    """Integrate every cluster over one soft step.  Returns
    (pos_new, vel_new, e0, e1, nsteps, status); dt_hard (n,), if given, is
    updated in place with each particle's last hard step."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n)).copy()
    vel = _f64(vel, (3, n)).copy()
    r_out = _f64(r_out, (n,))
    cl_ptr = np.ascontiguousarray(cl_ptr, dtype=np.int32)
    members = np.ascontiguousarray(members, dtype=np.int32)
    nc = cl_ptr.shape[0] - 1
    e0, e1 = np.empty(nc), np.empty(nc)
    ns = np.empty(nc, dtype=np.int64)
    pc = p.c()
    dt = p.dt_soft if dt_soft is None else float(dt_soft)
    dh = None
    if dt_hard is not None:
        if not (isinstance(dt_hard, np.ndarray) and dt_hard.dtype == np.float64 and dt_hard.shape == (n,)
                and dt_hard.flags.c_contiguous):
            raise ValueError("dt_hard must be a contiguous float64 (n,) array")
        dh = _d(dt_hard)
    st = lib().orc_hermite_clusters(n, nc, _i32(cl_ptr), _i32(members), _d(pos), _d(vel), _d(mass),
                                    _d(r_out), C.byref(pc), dt, dh, _d(e0), _d(e1), _i64(ns))
    return pos, vel, e0, e1, ns, int(st)


# code units (G = M_sun = 1 au = 1): grams and centimetres per unit
GRAM = 1.0 / 1.989e33
CM = 1.0 / 1.495978707e13


def density_code(rho_cgs: float) -> float:
    """A density in g / cm^3 in solar masses per au^3."""
    return rho_cgs * GRAM / CM ** 3


def hermite_collide(pos, vel, mass, r_out, cl_ptr, members, p: Params, f: float, rho: float, dt_soft=None,
                    dt_hard=None):
    """Hard part with perfect-accretion collisions (Section 2.5.1), radius
    enhancement f, bulk density rho (code units).  Returns a dict: pos, vel,
    merged_into (n,) int32, eps (nc, 6), e0, e1, nsteps, ncoll, tcoll (ticks
    of dt_soft 2^-40), status.  dt_hard (n,), if given, is updated in place."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos = _f64(pos, (3, n)).copy()
    vel = _f64(vel, (3, n)).copy()
    r_out = _f64(r_out, (n,))
    cl_ptr = np.ascontiguousarray(cl_ptr, dtype=np.int32)
    members = np.ascontiguousarray(members, dtype=np.int32)
    nc = cl_ptr.shape[0] - 1
    merged = np.arange(n, dtype=np.int32)
    eps = np.zeros((nc, 6))
    e0, e1 = np.empty(nc), np.empty(nc)
    ns, nco, tco = (np.empty(nc, dtype=np.int64) for _ in range(3))
    pc = p.c()
    dt = p.dt_soft if dt_soft is None else float(dt_soft)
    dh = None
    if dt_hard is not None:
        if not (isinstance(dt_hard, np.ndarray) and dt_hard.dtype == np.float64 and dt_hard.shape == (n,)
                and dt_hard.flags.c_contiguous):
            raise ValueError("dt_hard must be a contiguous float64 (n,) array")
        dh = _d(dt_hard)
    st = lib().orc_hermite_collide_clusters(n, nc, _i32(cl_ptr), _i32(members), _d(pos), _d(vel), _d(mass),
                                            _d(r_out), C.byref(pc), dt, dh, float(f), float(rho), _i32(merged),
                                            _d(eps), _d(e0), _d(e1), _i64(ns), _i64(nco), _i64(tco))
    return dict(pos=pos, vel=vel, merged_into=merged, eps=eps, e0=e0, e1=e1, nsteps=ns, ncoll=nco, tcoll=tco,
                status=int(st))


# -- neighbours and clusters ----------------------------------------------------
def neighbour_rows(pos, vel, mass, r_out, r_search, p: Params, idx=None):
    """CSR (row_ptr int64 (ni+1,), col int32) of the neighbour rows of idx."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos, vel = _f64(pos, (3, n)), _f64(vel, (3, n))
    r_out, r_search = _f64(r_out, (n,)), _f64(r_search, (n,))
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    ni = idx.shape[0]
    row_ptr = np.zeros(ni + 1, dtype=np.int64)
    pc = p.c()
    col = np.zeros(1, dtype=np.int32)
    nnz = lib().orc_neighbour_rows(n, _d(pos), _d(vel), _d(mass), _d(r_out), _d(r_search), C.byref(pc), ni,
                                   _i64(idx), _i64(row_ptr), _i32(col), 0)
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    nnz2 = lib().orc_neighbour_rows(n, _d(pos), _d(vel), _d(mass), _d(r_out), _d(r_search), C.byref(pc), ni,
                                    _i64(idx), _i64(row_ptr), _i32(col), col.shape[0])
    assert nnz2 == nnz
    return row_ptr, col[:nnz]


def is_neighbour(pi, pj, p: Params) -> bool:
    """pi, pj: sequences (x, y, z, vx, vy, vz, m, r_out, r_search)."""
    a, b = _f64(pi, (9,)), _f64(pj, (9,))
    pc = p.c()
    return bool(lib().orc_is_neighbour(_d(a), _d(b), C.byref(pc)))


def labels(row_ptr, col):
    """Cluster index of every particle (Section 2.3 steps i-iii) and the
    number of sweeps."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = row_ptr.shape[0] - 1
    lab = np.empty(max(n, 1), dtype=np.int32)
    sweeps = lib().orc_labels(n, _i64(row_ptr), _i32(col if col.size else np.zeros(1, np.int32)), _i32(lab))
    return lab[:n], int(sweeps)


def cluster_csr(label):
    """Clusters as (cl_ptr, members): members sorted by (label, index)."""
    label = np.asarray(label)
    order = np.lexsort((np.arange(label.shape[0]), label))
    lab_sorted = label[order]
    starts = np.flatnonzero(np.r_[True, lab_sorted[1:] != lab_sorted[:-1]]) if label.size else np.zeros(0, int)
    cl_ptr = np.r_[starts, label.shape[0]].astype(np.int32)
    return cl_ptr, order.astype(np.int32)


# -- adjoint --------------------------------------------------------------------
def soft_adjoint(pos, mass, r_out, lam, p: Params):
    """(dL/dpos (3, n), dL/dm (n,)) for L = sum_i lam_i . a_soft,i."""
    mass = _f64(mass)
    n = mass.shape[0]
    pos, r_out, lam = _f64(pos, (3, n)), _f64(r_out, (n,)), _f64(lam, (3, n))
    gp, gm = np.empty((3, n)), np.empty(n)
    lib().orc_soft_adjoint(n, _d(pos), _d(mass), _d(r_out), p.G, p.gamma, _d(lam), _d(gp), _d(gm))
    return gp, gm
