"""Seeded synthetic planetesimal disks (input generation only).

This module is shared by the oracle tests and the GPU path as the single
source of inputs.  It holds none of the method's arithmetic (no cut-off
radii, no changeover functions, no forces, no neighbour tests, no
integrator): it draws orbital elements and masses with numpy's seeded
generator and converts elements to heliocentric Cartesian states.

Units: G = M_sun = 1, 1 au = 1, 1 yr = 2*pi (Section 3.1 of the paper).

Workload recipes follow the paper's initial conditions (Section 3.1):
surface density proportional to a^(-3/2), eccentricities and inclinations
with rms e = 2 rms i = 2h (h the reduced Hill radius), uniform angles.
The paper draws e and i from a "Gaussian distribution with dispersion"; the
non-negative magnitudes are drawn here from Rayleigh distributions with the
stated rms values (Rayleigh scale = rms / sqrt(2)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Disk",
    "reduced_hill",
    "make_disk",
    "workload",
    "dense_ring",
    "hermite_clusters",
    "sample_indices",
    "WORKLOADS",
]


@dataclass
class Disk:
    """Heliocentric state of a disk in structure-of-arrays layout.

    pos, vel: float64 arrays of shape (3, n) (rows x, y, z), C-contiguous.
    mass: float64 (n,).  a, e, inc: the drawn osculating elements (for
    checks only).
    """

    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    a: np.ndarray
    e: np.ndarray
    inc: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])


def reduced_hill(m: float) -> float:
    """h = (m / 3 M_sun)^(1/3) (Section 3.1)."""
    return (m / 3.0) ** (1.0 / 3.0)


def _kepler_E(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly from mean anomaly by Newton iteration (e < 1)."""
    E = M + e * np.sin(M)
    for _ in range(50):
        f = E - e * np.sin(E) - M
        fp = 1.0 - e * np.cos(E)
        dE = f / fp
        E = E - dE
        if np.max(np.abs(dE)) < 1e-15:
            break
    return E


def elements_to_state(a, e, inc, Omega, omega, M, mu=1.0):
    """Osculating elements -> heliocentric position and velocity, (3, n) each."""
    E = _kepler_E(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    nmot = np.sqrt(mu / a**3)
    xp = a * (cE - e)
    yp = a * b * sE
    den = 1.0 - e * cE
    vxp = -a * nmot * sE / den
    vyp = a * nmot * b * cE / den
    cO, sO = np.cos(Omega), np.sin(Omega)
    co, so = np.cos(omega), np.sin(omega)
    ci, si = np.cos(inc), np.sin(inc)
    # rotation R_z(Omega) R_x(inc) R_z(omega) applied to the perifocal frame
    r11 = cO * co - sO * so * ci
    r12 = -cO * so - sO * co * ci
    r21 = sO * co + cO * so * ci
    r22 = -sO * so + cO * co * ci
    r31 = so * si
    r32 = co * si
    pos = np.stack([r11 * xp + r12 * yp, r21 * xp + r22 * yp, r31 * xp + r32 * yp])
    vel = np.stack([r11 * vxp + r12 * vyp, r21 * vxp + r22 * vyp, r31 * vxp + r32 * vyp])
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel)


def _mass_law(rng, n, m_min, m_max, slope):
    """Inverse-CDF draw from dN/dm proportional to m^slope on [m_min, m_max]."""
    p = slope + 1.0
    u = rng.random(n)
    lo, hi = m_min**p, m_max**p
    return (lo + u * (hi - lo)) ** (1.0 / p)


def make_disk(
    n: int,
    a_in: float,
    a_out: float,
    seed: int,
    m_equal: float | None = None,
    m_min: float = 1e-10,
    m_max: float = 1e-8,
    slope: float = -2.5,
    h_mass: float | None = None,
    rms_e: float | None = None,
    rms_i: float | None = None,
) -> Disk:
    """Draw a seeded disk.

    Semi-major axes follow surface density a^(-3/2) (dN/da ~ a^(-1/2)),
    i.e. a = (sqrt(a_in) + u (sqrt(a_out) - sqrt(a_in)))^2.  Masses are equal
    (m_equal) or follow dN/dm ~ m^slope on [m_min, m_max].  rms e = 2h and
    rms i = h with h the reduced Hill radius of h_mass (default: the equal
    mass, else 1e-9), unless rms_e / rms_i are given.
    """
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    sa, sb = math.sqrt(a_in), math.sqrt(a_out)
    a = (sa + u * (sb - sa)) ** 2
    if m_equal is not None:
        mass = np.full(n, float(m_equal))
        href = reduced_hill(m_equal if h_mass is None else h_mass)
    else:
        mass = _mass_law(rng, n, m_min, m_max, slope)
        href = reduced_hill(1e-9 if h_mass is None else h_mass)
    if rms_e is None:
        rms_e = 2.0 * href
    if rms_i is None:
        rms_i = href
    e = rng.rayleigh(rms_e / math.sqrt(2.0), n)
    e = np.minimum(e, 0.9)
    inc = rng.rayleigh(rms_i / math.sqrt(2.0), n)
    Omega = rng.random(n) * 2 * math.pi
    omega = rng.random(n) * 2 * math.pi
    M = rng.random(n) * 2 * math.pi
    pos, vel = elements_to_state(a, e, inc, Omega, omega, M)
    return Disk(pos, vel, np.ascontiguousarray(mass), a, e, inc,
                meta=dict(n=n, a_in=a_in, a_out=a_out, seed=seed, m_equal=m_equal,
                          rms_e=rms_e, rms_i=rms_i))


# Workloads: sizes, radial ranges, mass laws and seeds of the five
# benchmark configurations (see the design notes for the recipe).
WORKLOADS = {
    "disk2k_equal": dict(n=2048, a_in=0.9, a_out=1.1, seed=1, m_equal=1e-9),
    "disk64k_masslaw": dict(n=65536, a_in=0.5, a_out=1.5, seed=2),
    "disk1m_masslaw": dict(n=1 << 20, a_in=0.5, a_out=5.0, seed=3),
    "disk256k_masslaw": dict(n=262144, a_in=0.5, a_out=1.5, seed=5),
}


def workload(name: str, n: int | None = None) -> Disk:
    """A named workload disk; n overrides the size with the same recipe."""
    kw = dict(WORKLOADS[name])
    if n is not None:
        kw["n"] = int(n)
    return make_disk(**kw)


def dense_ring(n: int = 4096, seed: int = 11, width: float = 0.002, m: float = 1e-9) -> Disk:
    """A very dense narrow ring (a in [1 - width/2, 1 + width/2]) that yields
    thousands of close pairs: stresses the changeover region and the
    neighbour test in all of its branches."""
    return make_disk(n, 1.0 - width / 2, 1.0 + width / 2, seed, m_equal=m)


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct sorted indices in [0, n) (seeded)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def hermite_clusters(
    disk: Disk,
    n_clusters: int = 20000,
    seed: int = 4,
    median: float = 4.0,
    sigma: float = 1.1,
    n_max: int = 256,
    r_out: np.ndarray | None = None,
    compact: float | None = None,
):
    """Independent neighbour clusters drawn from a disk's neighbourhoods.

    Sizes: clamp(round(exp(N(ln median, sigma^2))), 1, n_max), the largest
    draw set to n_max.  Members: a random seed particle and its n-1 nearest
    neighbours (3-D).  Each cluster's members are copied into a fresh
    contiguous particle array (clusters may share disk particles), so the
    result is (pos, vel, mass, idx, cl_ptr) with cl_ptr the cluster offsets.

    compact: if given with r_out (the disk's cut-off radii, an input), each
    cluster's positions and velocities relative to its centre of mass are
    scaled so that the median nearest-member distance becomes compact *
    (median r_out of the cluster); this pushes members into the changeover
    region.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    sizes = np.clip(np.rint(np.exp(rng.normal(math.log(median), sigma, n_clusters))), 1, n_max)
    sizes = sizes.astype(np.int64)
    sizes[int(np.argmax(sizes))] = n_max
    seeds = rng.integers(0, disk.n, n_clusters)
    tree = cKDTree(disk.pos.T)
    members = []
    for s, k in zip(seeds, sizes):
        if k == 1:
            members.append(np.array([s], dtype=np.int64))
        else:
            _, nb = tree.query(disk.pos[:, s], k=int(k))
            members.append(np.sort(np.asarray(nb, dtype=np.int64)))
    idx = np.concatenate(members)
    cl_ptr = np.zeros(n_clusters + 1, dtype=np.int32)
    cl_ptr[1:] = np.cumsum([len(mm) for mm in members])
    pos = np.ascontiguousarray(disk.pos[:, idx])
    vel = np.ascontiguousarray(disk.vel[:, idx])
    mass = np.ascontiguousarray(disk.mass[idx])
    ro = None if r_out is None else np.ascontiguousarray(r_out[idx])
    if compact is not None:
        if ro is None:
            raise ValueError("compact needs r_out")
        for c in range(n_clusters):
            a, b = cl_ptr[c], cl_ptr[c + 1]
            if b - a < 2:
                continue
            m = mass[a:b]
            xc = (pos[:, a:b] * m).sum(axis=1, keepdims=True) / m.sum()
            vc = (vel[:, a:b] * m).sum(axis=1, keepdims=True) / m.sum()
            d, _ = cKDTree(pos[:, a:b].T).query(pos[:, a:b].T, k=2)
            s = compact * float(np.median(ro[a:b])) / float(np.median(d[:, 1]))
            pos[:, a:b] = xc + s * (pos[:, a:b] - xc)
            vel[:, a:b] = vc + s * (vel[:, a:b] - vc)
    return dict(pos=pos, vel=vel, mass=mass, r_out=ro, idx=idx, cl_ptr=cl_ptr, sizes=sizes)
