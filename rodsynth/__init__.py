"""Seeded synthetic rod suspensions.

This module only prepares inputs: rod centres, orientations (as unit
quaternions), lengths and external forces/torques, plus the periodic box that
a target volume fraction implies.  It holds none of the method's arithmetic
(no directors from quaternions, mobilities, constraint geometry or solver
steps), so both the CPU oracle and the HIP library can be fed from it without
sharing any code.

The workloads follow the paper's filament suspensions (Section "Results":
viscosity 0.01 pN s/um^2, timestep 1e-4 s; filament diameter 25 nm) at the
sizes of the benchmark configurations below.  Units are um, s and pN.

Draw order for one system: centres, orientations, lengths, forces, each from
``numpy.random.Generator(PCG64(seed))``.

Dense workloads start from relaxed, overlap-free configurations (the paper
resolves the overlaps of its initial configurations before timing,
Results, "Polarity sorting in a spherical shell"): ``relaxed_system`` draws
a random placement (axes as unit vectors) and removes its overlaps by plain
geometric pushes (``_relax.c``, its own segment-separation routine, compiled
with gcc); the quaternions are built from the relaxed axes afterwards.  That
step only moves inputs and never feeds a value to either side; the tests
check its output against the oracle's own gaps.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
import subprocess
import threading
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_RELAX_SRC = os.path.join(_HERE, "_relax.c")
_RELAX_LIB = os.path.join(_HERE, "librelax.so")
_relax_lock = threading.Lock()
_relax = None

ETA = 0.01          # pN s / um^2  (Section "Results")
DT = 1.0e-4         # s
DIAM = 0.025        # um, filament diameter
CUTOFF = 0.05       # um, pair-search threshold on the surface gap
TOL = 1.0e-8        # complementarity residual


@dataclasses.dataclass
class RodSystem:
    """One periodic suspension.  Arrays are float64, row-major, host memory."""
    x: np.ndarray            # [n, 3] centres, inside [0, box)
    quat: np.ndarray         # [n, 4] unit quaternions [s, px, py, pz]
    length: np.ndarray       # [n] rod lengths
    force: np.ndarray        # [n, 6] external force (3) and torque (3)
    box: float
    diam: float = DIAM
    cutoff: float = CUTOFF
    eta: float = ETA
    dt: float = DT
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def uniform_length(self) -> Optional[float]:
        """The common length when all rods are equal, else None."""
        if self.n and np.all(self.length == self.length[0]):
            return float(self.length[0])
        return None


def spherocylinder_volume(length: np.ndarray, diam: float) -> np.ndarray:
    """Volume of a cylinder of the given length capped by two hemispheres."""
    return math.pi * diam * diam * length / 4.0 + math.pi * diam ** 3 / 6.0


def box_for_volume_fraction(length: np.ndarray, diam: float, phi: float) -> float:
    return float((spherocylinder_volume(length, diam).sum() / phi) ** (1.0 / 3.0))


def _isotropic_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-uniform rotations: a normalised 4-D Gaussian.  The rotated body
    axis is then uniform on the sphere."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _vmf_quaternions(rng: np.random.Generator, n: int, kappa: float) -> np.ndarray:
    """Rotations whose image of the body z axis follows a von Mises-Fisher law
    about z with concentration kappa, with a uniform twist about the rod's own
    axis.  cos(polar angle) is drawn by the inverse CDF of Wood (1994)."""
    u = rng.random(n)
    w = 1.0 + np.log(u + (1.0 - u) * np.exp(-2.0 * kappa)) / kappa
    w = np.clip(w, -1.0, 1.0)
    phi = rng.random(n) * 2.0 * math.pi
    twist = rng.random(n) * 2.0 * math.pi
    return _tilt_twist_quaternions(w, phi, twist)


def _tilt_twist_quaternions(w: np.ndarray, phi: np.ndarray, twist: np.ndarray) -> np.ndarray:
    """The rotation that turns the body z axis to polar cosine w and azimuth
    phi, after a turn by `twist` about body z."""
    beta = np.arccos(np.clip(w, -1.0, 1.0))
    # tilt: rotation by beta about the horizontal axis (-sin phi, cos phi, 0),
    # twist: rotation by `twist` about z; composed as tilt * twist.
    c1, s1 = np.cos(beta / 2), np.sin(beta / 2)
    ax, ay = -np.sin(phi), np.cos(phi)
    c2, s2 = np.cos(twist / 2), np.sin(twist / 2)
    q = np.empty((w.shape[0], 4))
    q[:, 0] = c1 * c2
    q[:, 1] = s1 * ax * c2 + s1 * ay * s2
    q[:, 2] = s1 * ay * c2 - s1 * ax * s2
    q[:, 3] = c1 * s2
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def make_system(n: int, *, seed: int, box: Optional[float] = None,
                phi: Optional[float] = None, length=1.0,
                orientation: str = "isotropic", kappa: float = 20.0,
                diam: float = DIAM, cutoff: float = CUTOFF, eta: float = ETA,
                dt: float = DT, force_scale: float = 1.0, name: str = "") -> RodSystem:
    """Draw one suspension.  ``length`` is a number or a (lo, hi) uniform
    range; give either ``box`` or the volume fraction ``phi``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    # lengths are needed for the box before centres are placed, but are drawn
    # from their own stream so the documented draw order of the main stream
    # (centres, orientations, forces) does not depend on the length law.
    lrng = np.random.Generator(np.random.PCG64([seed, 1]))
    if isinstance(length, (tuple, list)):
        lens = lrng.uniform(length[0], length[1], n)
    else:
        lens = np.full(n, float(length))
    if box is None:
        if phi is None:
            raise ValueError("give box or phi")
        box = box_for_volume_fraction(lens, diam, phi)
    x = rng.random((n, 3)) * box
    x = np.where(x >= box, 0.0, x)
    if orientation == "isotropic":
        quat = _isotropic_quaternions(rng, n)
    elif orientation == "vmf":
        quat = _vmf_quaternions(rng, n, kappa)
    else:
        raise ValueError(orientation)
    force = rng.standard_normal((n, 6)) * force_scale
    return RodSystem(x=np.ascontiguousarray(x), quat=np.ascontiguousarray(quat),
                     length=lens, force=np.ascontiguousarray(force), box=float(box),
                     diam=diam, cutoff=cutoff, eta=eta, dt=dt, name=name)


# --- overlap-free placements ---------------------------------------------------

def build_relax(force: bool = True) -> str:
    """Compile the overlap-removal routine (plain C, OpenMP)."""
    if force or not os.path.exists(_RELAX_LIB):
        tmp = _RELAX_LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _RELAX_SRC, "-lm"],
                       check=True)
        os.replace(tmp, _RELAX_LIB)
    return _RELAX_LIB


def _relax_lib():
    global _relax
    with _relax_lock:
        if _relax is None:
            if not os.path.exists(_RELAX_LIB) or os.path.getmtime(_RELAX_LIB) < os.path.getmtime(_RELAX_SRC):
                build_relax(force=True)
            lib = C.CDLL(_RELAX_LIB)
            lib.rs_relax.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                     C.c_double, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_double)]
            lib.rs_relax.restype = C.c_int
            _relax = lib
    return _relax


class RelaxError(RuntimeError):
    pass


def _cpu_threads() -> int:
    """Threads for the relaxation: OMP_NUM_THREADS if set, else the CPUs this
    process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def relaxed_system(n: int, *, seed: int, phi: float, length=1.0, diam: float = DIAM,
                   cutoff: float = CUTOFF, eta: float = ETA, dt: float = DT, gap: float = 3e-4,
                   gap_min: float = 1e-4, max_sweeps: int = 2000, force_scale: float = 1.0,
                   threads: int = 0, name: str = "") -> RodSystem:
    """An isotropic suspension at volume fraction ``phi`` with every pair of
    rods (and periodic images) separated by more than ``gap_min`` beyond
    contact.  Draw order from ``PCG64(seed)``: centres, axes (normalised
    Gaussian 3-vectors), twists, forces; lengths from ``PCG64([seed, 1])``
    as in ``make_system``.  The centres and axes are then relaxed; the
    quaternion of each rod turns body z to its relaxed axis after its twist."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lrng = np.random.Generator(np.random.PCG64([seed, 1]))
    if isinstance(length, (tuple, list)):
        lens = lrng.uniform(length[0], length[1], n)
    else:
        lens = np.full(n, float(length))
    box = box_for_volume_fraction(lens, diam, phi)
    x = rng.random((n, 3)) * box
    x = np.ascontiguousarray(np.where(x >= box, 0.0, x))
    ax = rng.standard_normal((n, 3))
    ax = np.ascontiguousarray(ax / np.linalg.norm(ax, axis=1, keepdims=True))
    twist = rng.random(n) * 2.0 * math.pi
    force = np.ascontiguousarray(rng.standard_normal((n, 6)) * force_scale)
    lens = np.ascontiguousarray(lens)
    boxv = np.full(3, box)
    worst = C.c_double(0.0)
    p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    nthreads = threads if threads > 0 else _cpu_threads()
    sweeps = _relax_lib().rs_relax(n, p(x), p(ax), p(lens), p(boxv), diam, gap, gap_min, max_sweeps, nthreads,
                                   C.byref(worst))
    if os.environ.get("RODSYNTH_VERBOSE"):
        print(f"relaxed_system: {sweeps} sweeps, smallest gap {worst.value:.3g}", flush=True)
    if sweeps < 0:
        raise RelaxError(f"overlaps not removed after {max_sweeps} sweeps (smallest gap {worst.value:.3g})")
    quat = _tilt_twist_quaternions(ax[:, 2], np.arctan2(ax[:, 1], ax[:, 0]), twist)
    return RodSystem(x=x, quat=np.ascontiguousarray(quat), length=lens, force=force, box=float(box),
                     diam=diam, cutoff=cutoff, eta=eta, dt=dt, name=name)


# --- the benchmark workloads -------------------------------------------------

def cfg_small(seed: int = 0) -> RodSystem:
    """1,000 rods of length 1 in a periodic cube of side 4, isotropic."""
    return make_system(1000, seed=seed, box=4.0, orientation="isotropic",
                       name="rods1k_box4_iso")


def cfg_paper_scale(seed: int = 0, n: int = 100_000) -> RodSystem:
    """100,000 rods of length 1, volume fraction 0.05, nematic (vMF kappa=20
    about z).  ``n`` may be lowered for a scaled-down copy at the same
    density."""
    return make_system(n, seed=seed, phi=0.05, orientation="vmf", kappa=20.0,
                       name=f"rods{n // 1000}k_phi0.05_vmf20")


def cfg_precision(seed: int = 0, n: int = 400_000, phi: float = 0.08, relaxed: bool = True) -> RodSystem:
    """400,000 rods, lengths uniform in [0.5, 1.5], isotropic, volume
    fraction 0.08, from a relaxed (overlap-free) start.  Random placements
    this dense overlap in self-stressed clusters whose linearised problem has
    no solution (a non-negative D d = 0 with phi.d < 0 exists); with every
    gap non-negative it always has one.  relaxed=False gives the raw random
    placement (``make_system``)."""
    name = f"rods{n // 1000}k_phi{phi}_iso_L0.5-1.5" + ("_relaxed" if relaxed else "")
    if relaxed:
        return relaxed_system(n, seed=seed, phi=phi, length=(0.5, 1.5), name=name)
    return make_system(n, seed=seed, phi=phi, length=(0.5, 1.5), orientation="isotropic", name=name)


def batch_plan(seed: int = 0, systems: int = 256, n_lo: int = 200, n_hi: int = 20_000, phi_range=(0.02, 0.1)):
    """Rod counts (log-uniform in [n_lo, n_hi]) and volume fractions (uniform
    in phi_range) of the batch, from PCG64([seed, 7])."""
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    counts = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), systems))).astype(int)
    phis = rng.uniform(phi_range[0], phi_range[1], systems)
    return counts, phis


def cfg_batched(seed: int = 0, systems: int = 256, n_lo: int = 200, n_hi: int = 20_000,
                phi_range=(0.02, 0.1), relaxed: bool = True, workers: int = 0) -> List[RodSystem]:
    """Independent periodic systems of rods of length 1, isotropic, rod
    counts log-uniform in [n_lo, n_hi], volume fractions uniform in
    phi_range; system k uses seed * 100003 + k.  Each starts relaxed
    (overlap-free, as ``cfg_precision``); the systems are relaxed
    concurrently on ``workers`` threads (0: the CPUs available)."""
    counts, phis = batch_plan(seed, systems, n_lo, n_hi, phi_range)
    if not relaxed:
        return [make_system(int(c), seed=seed * 100_003 + k, phi=float(p), orientation="isotropic",
                            name=f"batch{k}") for k, (c, p) in enumerate(zip(counts, phis))]
    from concurrent.futures import ThreadPoolExecutor
    nw = workers if workers > 0 else _cpu_threads()

    def one(k):
        return relaxed_system(int(counts[k]), seed=seed * 100_003 + k, phi=float(phis[k]), threads=1,
                              name=f"batch{k}")

    # largest systems first, so that the pool ends together
    order = sorted(range(systems), key=lambda k: -int(counts[k]))
    with ThreadPoolExecutor(max_workers=nw) as pool:
        done = dict(zip(order, pool.map(one, order)))
    return [done[k] for k in range(systems)]


def cfg_rollout(seed: int = 0, n: int = 50_000) -> RodSystem:
    """50,000 rods of length 1, volume fraction 0.05, isotropic."""
    return make_system(n, seed=seed, phi=0.05, orientation="isotropic",
                       name=f"rods{n // 1000}k_phi0.05_iso")


def confined_system(n: int = 3200, *, seed: int = 0, radius: float = 3.0, length: float = 1.0,
                    margin: float = 0.02, diam: float = DIAM, force_scale: float = 1.0,
                    name: str = "") -> RodSystem:
    """Rods of one length inside a spherical shell (the paper's confined
    suspension: 3,200 microtubules 1 um long in a sphere of radius 3 um,
    Fig. 1).  Centres uniform in the ball and axes isotropic, redrawn until
    both ends lie at least `margin` + diam/2 inside the shell; the periodic
    box is wide enough that no rod meets another's image.  Draw order from
    PCG64(seed): rounds of (centres, axes, twists) for the rods still
    outside, then forces."""
    rng = np.random.Generator(np.random.PCG64(seed))
    box = 2.0 * radius + 2.0 * length + 1.0
    c = np.full(3, 0.5 * box)
    x = np.empty((n, 3))
    ax = np.empty((n, 3))
    tw = np.empty(n)
    todo = np.arange(n)
    lim = radius - margin - 0.5 * diam
    while todo.size:
        m = todo.size
        xc = c + radius * (rng.random((m, 3)) * 2.0 - 1.0)
        a = rng.standard_normal((m, 3))
        a /= np.linalg.norm(a, axis=1, keepdims=True)
        t = rng.random(m) * 2.0 * math.pi
        ok = (np.linalg.norm(xc + 0.5 * length * a - c, axis=1) <= lim) & \
             (np.linalg.norm(xc - 0.5 * length * a - c, axis=1) <= lim)
        x[todo[ok]], ax[todo[ok]], tw[todo[ok]] = xc[ok], a[ok], t[ok]
        todo = todo[~ok]
    quat = _tilt_twist_quaternions(ax[:, 2], np.arctan2(ax[:, 1], ax[:, 0]), tw)
    force = rng.standard_normal((n, 6)) * force_scale
    return RodSystem(x=np.ascontiguousarray(x), quat=np.ascontiguousarray(quat), length=np.full(n, float(length)),
                     force=np.ascontiguousarray(force), box=float(box), diam=diam,
                     name=name or f"rods{n}_sphere_r{radius}")


def shell_wall(s: RodSystem, radius: float = 3.0):
    """The spherical shell of ``confined_system`` as (kind, p, a, r) with
    kind 1 (rods inside)."""
    c = 0.5 * s.box
    return (1, (c, c, c), (0.0, 0.0, 1.0), float(radius))


def cfg_hub(seed: int = 0, crossers: int = 36) -> RodSystem:
    """One long rod (length 4, along x) crossed by ``crossers`` short rods
    (length 1, along y with small tilts) whose axes pass 0.005-0.06 um above
    it: the long rod takes part in ``crossers`` constraints, half with a
    lower and half with a higher index, so both of its incidence lists are
    long.  Box 10; forces N(0, 1), with 2 pN more along -z on every crosser
    (pressing it onto the long rod).  Draw order: offsets along z, tilts,
    forces."""
    rng = np.random.Generator(np.random.PCG64([seed, 11]))
    n = crossers + 1
    hub = crossers // 2
    x = np.empty((n, 3))
    quat = np.empty((n, 4))
    lens = np.ones(n)
    off = rng.uniform(0.005, 0.06, crossers)
    tilt = rng.uniform(-0.05, 0.05, (crossers, 2))
    force = rng.standard_normal((n, 6))
    h = math.sqrt(0.5)
    # hub: the rotation by +90 degrees about y (z -> x)
    x[hub] = (5.0, 5.0, 5.0)
    quat[hub] = (h, 0.0, h, 0.0)
    lens[hub] = 4.0
    k = 0
    for m in range(crossers):
        i = m if m < hub else m + 1
        x[i] = (3.25 + 0.1 * m, 5.0, 5.0 + off[k])
        # -90 degrees about x (z -> y), then a small extra turn about x and z
        a, b = tilt[k]
        qx = np.array([math.cos(-math.pi / 4 + a / 2), math.sin(-math.pi / 4 + a / 2), 0.0, 0.0])
        qz = np.array([math.cos(b / 2), 0.0, 0.0, math.sin(b / 2)])
        # Hamilton product qz * qx
        s1, v1 = qz[0], qz[1:]
        s2, v2 = qx[0], qx[1:]
        qv = np.concatenate([[s1 * s2 - v1 @ v2], s1 * v2 + s2 * v1 + np.cross(v1, v2)])
        quat[i] = qv / np.linalg.norm(qv)
        force[i, 2] -= 2.0
        k += 1
    return RodSystem(x=x, quat=quat, length=lens, force=force, box=10.0, name="hub")


# --- crosslinkers ---------------------------------------------------------------

def crosslinker_positions(m: int, box: float, seed: int = 0) -> np.ndarray:
    """m unbound crosslinkers uniform in the periodic box, from
    PCG64([seed, 12])."""
    rng = np.random.Generator(np.random.PCG64([seed, 12]))
    x = rng.random((m, 3)) * box
    return np.ascontiguousarray(np.where(x >= box, 0.0, x))


def crosslinker_positions_ball(m: int, centre, radius: float, seed: int = 0) -> np.ndarray:
    """m unbound crosslinkers uniform in a ball (a confined suspension's
    shell), by rejection from its bounding cube, from PCG64([seed, 14])."""
    rng = np.random.Generator(np.random.PCG64([seed, 14]))
    c = np.asarray(centre, dtype=np.float64)
    out = np.empty((m, 3))
    k = 0
    while k < m:
        y = c + radius * (rng.random((2 * (m - k) + 16, 3)) * 2.0 - 1.0)
        y = y[np.linalg.norm(y - c, axis=1) <= radius][: m - k]
        out[k:k + len(y)] = y
        k += len(y)
    return np.ascontiguousarray(out)


def kmc_draws(m: int, seed: int, step: int):
    """The random numbers of one kinetics step: u[m][4] uniform in [0, 1) and
    xi[m][3] standard normal, from PCG64([seed, 13, step])."""
    rng = np.random.Generator(np.random.PCG64([seed, 13, step]))
    u = rng.random((m, 4))
    xi = rng.standard_normal((m, 3))
    return np.ascontiguousarray(u), np.ascontiguousarray(xi)
