"""CPU FP64 oracle for the steric-constraint step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product library never does.  It
shares no code with the HIP library.  The arithmetic lives in
``rodlcp_oracle.c`` (plain sequential C, double precision); this file only
marshals numpy arrays.  ``crosscheck.py`` adds dense cross-check solvers for
tiny systems.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rodlcp_oracle.c")
_SRC_KMC = os.path.join(_HERE, "kmc_oracle.c")
_SOURCES = (_SRC, _SRC_KMC)
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

IMG_ZERO = 0x888
FLAG_CUTOFF, FLAG_PARALLEL, FLAG_DEGENERATE = 1, 2, 4
OK, NOT_CONVERGED, STAGNATED = 0, 1, 2


_CHECK_FLAGS = ["-O2", "-ffp-contract=off"]
# Timing build of the same source for the CPU baseline: optimised for the
# host it runs on, so it is compiled there, into a private temporary folder,
# and never loaded by the tests' checker calls.
_TIMING_FLAGS = ["-O3", "-march=native"]
_timing_lib = None
_active = "check"


def _compile(out: str, flags) -> None:
    tmp = out + ".tmp"
    cmd = ["gcc", *flags, "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp, *_SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB):
        _compile(_LIB, _CHECK_FLAGS)
    return _LIB


def use_build(name: str) -> str:
    """Select the library the wrappers call: "check" (the default, -O2
    -ffp-contract=off, what every test uses) or "timing" (-O3 -march=native,
    built on first use for this host; the same source, so its results agree
    with the checker's to rounding).  Returns the previous choice."""
    global _active
    if name not in ("check", "timing"):
        raise ValueError(name)
    prev, _active = _active, name
    return prev


def _load():
    global _lib, _timing_lib
    with _lock:
        if _active == "timing":
            if _timing_lib is None:
                import tempfile
                out = os.path.join(tempfile.mkdtemp(prefix="rodlcp_oracle_"), "liboracle_timing.so")
                _compile(out, _TIMING_FLAGS)
                _timing_lib = _declare(C.CDLL(out))
            return _timing_lib
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SOURCES):
                build(force=True)
            _lib = _declare(C.CDLL(_LIB))
    return _lib


def _declare(lib):
    """Argument and result types of the exported functions."""
    P = C.c_void_p
    I64 = C.c_int64
    D = C.c_double
    lib.ora_img_pack.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.ora_img_pack.restype = C.c_int
    lib.ora_rotation.argtypes = [P, P]
    lib.ora_directors.argtypes = [I64, P, P]
    lib.ora_psi_times.argtypes = [P, P, P]
    lib.ora_mobility_coeffs.argtypes = [D, D, D, P]
    lib.ora_mobility_block.argtypes = [P, D, D, D, P]
    lib.ora_apply_mobility.argtypes = [I64, P, P, D, D, D, P, P]
    lib.ora_closest_flat.argtypes = [P, P, D, P, P, D, P]
    for fn in (lib.ora_pairs_brute, lib.ora_pairs_cells):
        fn.argtypes = [I64, P, P, P, D, P, D, D, I64, P, P, P, P]
        fn.restype = I64
    lib.ora_assemble.argtypes = [I64, P, P, P, D, P, D, D, D, I64, P, P, P, P, P, P, P, P]
    lib.ora_dense_D.argtypes = [I64, P, I64, P, P, P, P, P]
    lib.ora_apply_Mc.argtypes = [I64, P, P, D, D, D, I64, P, P, P, P, P, P, P]
    lib.ora_velocity.argtypes = [I64, P, P, D, D, D, I64, P, P, P, P, P, P, P]
    lib.ora_bbpgd.argtypes = [I64, P, P, D, D, D, I64, P, P, P, P, P, D, I64, P, P, P]
    lib.ora_bbpgd.restype = C.c_int
    lib.ora_integrate.argtypes = [I64, P, D, P, P, P, P]
    lib.ora_bbpgd_gen.argtypes = [I64, P, P, D, D, D, I64, P, P, P, P, P, P, P, D, I64, P, P, P]
    lib.ora_bbpgd_gen.restype = C.c_int
    lib.ora_apply_Mc_gen.argtypes = [I64, P, P, D, D, D, I64, P, P, P, P, P, P, P, P, P]
    lib.ora_links.argtypes = [I64, P, P, P, D, P, D, D, D, I64, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.ora_walls.argtypes = [I64, P, P, P, D, D, D, D, D, I64, P, P, I64, P, P, P, P, P]
    lib.ora_walls.restype = I64
    lib.ora_mobility_pow_block.argtypes = [P, D, D, D, D, P]
    lib.ora_brownian_force.argtypes = [I64, P, P, D, D, D, D, D, P, P]
    lib.ora_kmc_effective_volume.argtypes = [P]
    lib.ora_kmc_effective_volume.restype = D
    lib.ora_kmc_inside_length.argtypes = [I64, P, P, P, D, P, I64, P, D]
    lib.ora_kmc_inside_length.restype = D
    lib.ora_kmc_cross_sum.argtypes = [I64, P, P, P, D, P, P, P, I64]
    lib.ora_kmc_cross_sum.restype = D
    lib.ora_kmc_step.argtypes = [I64, P, P, P, D, P, P, D, I64, P, P, P, P, P, P, P]
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _len_args(length, n):
    """(len array or None, uniform length)."""
    if length is None:
        raise ValueError("length required")
    if np.isscalar(length):
        return None, float(length)
    arr = _f64(length)
    if arr.shape != (n,):
        raise ValueError("length shape")
    return arr, 0.0


def _box3(box) -> np.ndarray:
    b = np.asarray(box, dtype=np.float64).reshape(-1)
    return _f64(np.repeat(b, 3) if b.size == 1 else b)


# --- geometry ----------------------------------------------------------------

def img_pack(nx: int, ny: int, nz: int) -> int:
    return int(_load().ora_img_pack(nx, ny, nz))


def img_unpack(img) -> np.ndarray:
    img = np.asarray(img, dtype=np.int64)
    return np.stack([((img >> 8) & 15) - 8, ((img >> 4) & 15) - 8, (img & 15) - 8], axis=-1)


def rotation(quat) -> np.ndarray:
    q = _f64(quat)
    R = np.empty(9)
    _load().ora_rotation(_p(q), _p(R))
    return R.reshape(3, 3)


def directors(quat) -> np.ndarray:
    q = _f64(quat)
    n = q.shape[0]
    d = np.empty((n, 3))
    _load().ora_directors(n, _p(q), _p(d))
    return d


def psi_times(quat, omega) -> np.ndarray:
    q, w = _f64(quat), _f64(omega)
    out = np.empty(4)
    _load().ora_psi_times(_p(q), _p(w), _p(out))
    return out


def mobility_coeffs(L: float, diam: float, eta: float) -> np.ndarray:
    c = np.empty(4)
    _load().ora_mobility_coeffs(L, diam, eta, _p(c))
    return c


def mobility_block(d, L: float, diam: float, eta: float) -> np.ndarray:
    dd = _f64(d)
    M = np.empty(36)
    _load().ora_mobility_block(_p(dd), L, diam, eta, _p(M))
    return M.reshape(6, 6)


def apply_mobility(dir_, length, diam, eta, F) -> np.ndarray:
    d = _f64(dir_)
    n = d.shape[0]
    la, l0 = _len_args(length, n)
    Fa = _f64(F)
    U = np.empty((n, 6))
    _load().ora_apply_mobility(n, _p(d), _p(la), l0, diam, eta, _p(Fa), _p(U))
    return U


def closest(xi, di, Li, xj, dj, Lj):
    """Closest points of two rod axes: (s, t, dist, e[3], flags)."""
    out = np.empty(7)
    a = [_f64(v) for v in (xi, di, xj, dj)]
    _load().ora_closest_flat(_p(a[0]), _p(a[1]), float(Li), _p(a[2]), _p(a[3]), float(Lj), _p(out))
    return out[0], out[1], out[2], out[3:6].copy(), int(out[6])


@dataclass
class Pairs:
    pi: np.ndarray
    pj: np.ndarray
    img: np.ndarray
    flags: np.ndarray

    @property
    def n(self) -> int:
        return int(self.pi.shape[0])


def pairs(x, dir_, length, box, diam, cutoff, method: str = "auto") -> Pairs:
    """Canonical near-contact pair list; 'brute' is the definition, 'cells'
    an independent uniform-grid search (used for large n)."""
    xa, d = _f64(x), _f64(dir_)
    n = xa.shape[0]
    la, l0 = _len_args(length, n)
    b = _box3(box)
    lib = _load()
    if method == "auto":
        method = "brute" if n <= 3000 else "cells"
    fn = lib.ora_pairs_brute if method == "brute" else lib.ora_pairs_cells
    cap = 16 * n + 64
    while True:
        pi = np.empty(cap, np.int32)
        pj = np.empty(cap, np.int32)
        img = np.empty(cap, np.int32)
        fl = np.empty(cap, np.uint8)
        cnt = fn(n, _p(xa), _p(d), _p(la), l0, _p(b), diam, cutoff, cap, _p(pi), _p(pj), _p(img), _p(fl))
        if cnt <= cap:
            return Pairs(pi[:cnt].copy(), pj[:cnt].copy(), img[:cnt].copy(), fl[:cnt].copy())
        cap = int(cnt)


@dataclass
class Constraints:
    phi: np.ndarray   # [nc]
    e: np.ndarray     # [nc, 3]
    arm: np.ndarray   # [nc, 2]
    q: np.ndarray     # [nc]


def assemble(x, dir_, length, box, diam, eta, dt, pr: Pairs, F) -> Constraints:
    xa, d, Fa = _f64(x), _f64(dir_), _f64(F)
    n = xa.shape[0]
    la, l0 = _len_args(length, n)
    b = _box3(box)
    nc = pr.n
    phi, q = np.empty(nc), np.empty(nc)
    e, arm = np.empty((nc, 3)), np.empty((nc, 2))
    pi, pj, img = _i32(pr.pi), _i32(pr.pj), _i32(pr.img)
    _load().ora_assemble(n, _p(xa), _p(d), _p(la), l0, _p(b), diam, eta, dt, nc, _p(pi), _p(pj), _p(img),
                         _p(Fa), _p(phi), _p(e), _p(arm), _p(q))
    return Constraints(phi, e, arm, q)


def dense_D(dir_, pr: Pairs, cs: Constraints) -> np.ndarray:
    d = _f64(dir_)
    n, nc = d.shape[0], pr.n
    D = np.empty((6 * n, nc))
    _load().ora_dense_D(n, _p(d), nc, _p(_i32(pr.pi)), _p(_i32(pr.pj)), _p(_f64(cs.e)), _p(_f64(cs.arm)), _p(D))
    return D


def apply_Mc(dir_, length, diam, eta, pr: Pairs, cs: Constraints, gamma, add_q: bool = True) -> np.ndarray:
    d = _f64(dir_)
    n, nc = d.shape[0], pr.n
    la, l0 = _len_args(length, n)
    g = _f64(gamma)
    w = np.empty(nc)
    q = _f64(cs.q) if add_q else None
    _load().ora_apply_Mc(n, _p(d), _p(la), l0, diam, eta, nc, _p(_i32(pr.pi)), _p(_i32(pr.pj)),
                         _p(_f64(cs.e)), _p(_f64(cs.arm)), _p(q), _p(g), _p(w))
    return w


def velocity(dir_, length, diam, eta, pr: Pairs, cs: Constraints, gamma, F) -> np.ndarray:
    d = _f64(dir_)
    n, nc = d.shape[0], pr.n
    la, l0 = _len_args(length, n)
    U = np.empty((n, 6))
    _load().ora_velocity(n, _p(d), _p(la), l0, diam, eta, nc, _p(_i32(pr.pi)), _p(_i32(pr.pj)),
                         _p(_f64(cs.e)), _p(_f64(cs.arm)), _p(_f64(gamma)), _p(_f64(F)), _p(U))
    return U


@dataclass
class SolveResult:
    gamma: np.ndarray
    g: np.ndarray
    iterations: int
    residual: float
    alpha0: float
    status: int


def bbpgd(dir_, length, diam, eta, pr: Pairs, cs: Constraints, tol=1e-8, max_iter=100_000,
          gamma0=None) -> SolveResult:
    d = _f64(dir_)
    n, nc = d.shape[0], pr.n
    la, l0 = _len_args(length, n)
    gamma = np.zeros(nc) if gamma0 is None else _f64(gamma0).copy()
    g = np.empty(nc)
    info = np.zeros(3)
    st = _load().ora_bbpgd(n, _p(d), _p(la), l0, diam, eta, nc, _p(_i32(pr.pi)), _p(_i32(pr.pj)),
                           _p(_f64(cs.e)), _p(_f64(cs.arm)), _p(_f64(cs.q)), tol, int(max_iter),
                           _p(gamma), _p(g), _p(info))
    return SolveResult(gamma, g, int(info[0]), float(info[1]), float(info[2]), int(st))


def integrate(box, dt, U, x, quat, xu=None):
    """In place: x, quat (and xu if given) advance by one step."""
    b = _box3(box)
    n = x.shape[0]
    for a in (U, x, quat) + ((xu,) if xu is not None else ()):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().ora_integrate(n, _p(b), float(dt), _p(U), _p(x), _p(xu), _p(quat))


# --- one whole step ------------------------------------------------------------

@dataclass
class StepResult:
    dir: np.ndarray
    pairs: Pairs
    cons: Constraints
    solve: SolveResult
    U: np.ndarray


def step_solve(sys, tol=None, max_iter=100_000, pair_method="auto") -> StepResult:
    """Directors, pairs, constraint geometry, BBPGD and U for one rod system
    (an object with x, quat, length, force, box, diam, cutoff, eta, dt)."""
    tol = 1e-8 if tol is None else tol
    d = directors(sys.quat)
    L = sys.uniform_length if sys.uniform_length is not None else sys.length
    pr = pairs(sys.x, d, L, sys.box, sys.diam, sys.cutoff, method=pair_method)
    cs = assemble(sys.x, d, L, sys.box, sys.diam, sys.eta, sys.dt, pr, sys.force)
    sr = bbpgd(d, L, sys.diam, sys.eta, pr, cs, tol=tol, max_iter=max_iter)
    U = velocity(d, L, sys.diam, sys.eta, pr, cs, sr.gamma, sys.force)
    return StepResult(d, pr, cs, sr, U)


# --- bilateral links and general constraint sets ------------------------------

@dataclass
class Links:
    """Hookean links between points on two rod axes (q < 0: to a fixed point)."""
    p: np.ndarray        # [nl] int32
    q: np.ndarray        # [nl] int32, -1 for a link to anchor[k]
    arm: np.ndarray      # [nl, 2] arclengths (sP, sQ)
    kappa: np.ndarray    # [nl] stiffness, +inf for a rigid joint
    rest: np.ndarray     # [nl] rest length
    anchor: Optional[np.ndarray] = None  # [nl, 3]

    @property
    def n(self) -> int:
        return int(self.p.shape[0])


@dataclass
class LinkGeometry:
    length: np.ndarray   # [nl]
    e: np.ndarray        # [nl, 3]
    q: np.ndarray        # [nl]
    cmp: np.ndarray      # [nl] compliance 1/(kappa h)
    flags: np.ndarray    # [nl] uint8


def links_geometry(x, dir_, length, box, diam, eta, dt, lk: Links, F=None) -> LinkGeometry:
    xa, d = _f64(x), _f64(dir_)
    n = xa.shape[0]
    la, l0 = _len_args(length, n)
    nl = lk.n
    out = LinkGeometry(np.empty(nl), np.empty((nl, 3)), np.empty(nl), np.empty(nl), np.empty(nl, np.uint8))
    anchor = _f64(lk.anchor) if lk.anchor is not None else None
    _load().ora_links(n, _p(xa), _p(d), _p(la), l0, _p(_box3(box)), diam, eta, dt, nl, _p(_i32(lk.p)),
                      _p(_i32(lk.q)), _p(_f64(lk.arm)), _p(_f64(lk.kappa)), _p(_f64(lk.rest)), _p(anchor),
                      _p(None if F is None else _f64(F)), _p(out.length), _p(out.e), _p(out.q), _p(out.cmp),
                      _p(out.flags))
    return out


@dataclass
class General:
    """A general constraint list: contacts (kind 0) and links (kind 1); pj < 0
    for a constraint against a fixed body."""
    pi: np.ndarray
    pj: np.ndarray
    e: np.ndarray
    arm: np.ndarray
    q: np.ndarray
    kind: np.ndarray     # uint8
    cmp: np.ndarray

    @property
    def n(self) -> int:
        return int(self.pi.shape[0])


def general(pr: Optional[Pairs] = None, cs: Optional[Constraints] = None, lk: Optional[Links] = None,
            lg: Optional[LinkGeometry] = None) -> General:
    """Contacts first, then links, each in its own order."""
    parts = []
    if pr is not None and pr.n:
        parts.append((pr.pi, pr.pj, cs.e, cs.arm, cs.q, np.zeros(pr.n, np.uint8), np.zeros(pr.n)))
    if lk is not None and lk.n:
        parts.append((lk.p, lk.q, lg.e, lk.arm, lg.q, np.ones(lk.n, np.uint8), lg.cmp))
    if not parts:
        z = np.zeros(0)
        return General(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros((0, 2)), z,
                       np.zeros(0, np.uint8), z)
    cols = list(zip(*parts))
    return General(_i32(np.concatenate(cols[0])), _i32(np.concatenate(cols[1])), _f64(np.concatenate(cols[2])),
                   _f64(np.concatenate(cols[3])), _f64(np.concatenate(cols[4])),
                   np.ascontiguousarray(np.concatenate(cols[5]), dtype=np.uint8), _f64(np.concatenate(cols[6])))


def apply_Mc_gen(dir_, length, diam, eta, gc: General, gamma, add_q: bool = True) -> np.ndarray:
    d = _f64(dir_)
    n = d.shape[0]
    la, l0 = _len_args(length, n)
    w = np.empty(gc.n)
    _load().ora_apply_Mc_gen(n, _p(d), _p(la), l0, diam, eta, gc.n, _p(gc.pi), _p(gc.pj), _p(gc.e), _p(gc.arm),
                             _p(gc.q if add_q else None), _p(gc.kind), _p(gc.cmp), _p(_f64(gamma)), _p(w))
    return w


def bbpgd_gen(dir_, length, diam, eta, gc: General, tol=1e-8, max_iter=100_000, gamma0=None) -> SolveResult:
    d = _f64(dir_)
    n = d.shape[0]
    la, l0 = _len_args(length, n)
    gamma = np.zeros(gc.n) if gamma0 is None else _f64(gamma0).copy()
    g = np.empty(gc.n)
    info = np.zeros(3)
    st = _load().ora_bbpgd_gen(n, _p(d), _p(la), l0, diam, eta, gc.n, _p(gc.pi), _p(gc.pj), _p(gc.e), _p(gc.arm),
                               _p(gc.q), _p(gc.kind), _p(gc.cmp), tol, int(max_iter), _p(gamma), _p(g), _p(info))
    return SolveResult(gamma, g, int(info[0]), float(info[1]), float(info[2]), int(st))


def velocity_gen(dir_, length, diam, eta, gc: General, gamma, F) -> np.ndarray:
    """U = M (D gamma + F) over a general constraint list."""
    d = _f64(dir_)
    n = d.shape[0]
    la, l0 = _len_args(length, n)
    U = np.empty((n, 6))
    _load().ora_velocity(n, _p(d), _p(la), l0, diam, eta, gc.n, _p(gc.pi), _p(gc.pj), _p(gc.e), _p(gc.arm),
                         _p(_f64(gamma)), _p(_f64(F)), _p(U))
    return U


# --- walls ---------------------------------------------------------------------

WALL_PLANE, WALL_SPHERE_IN, WALL_CYLINDER_IN = 0, 1, 2


def wall(kind: int, p, a=(0.0, 0.0, 1.0), r: float = 0.0) -> np.ndarray:
    """One wall as 8 doubles {kind, p[3], a[3], r}."""
    return np.array([float(kind), *map(float, p), *map(float, a), float(r)])


@dataclass
class WallContacts:
    rod: np.ndarray    # [m] int32
    e: np.ndarray      # [m, 3] unit normal into the allowed region
    arm: np.ndarray    # [m, 2] (s, 0)
    phi: np.ndarray    # [m]
    q: np.ndarray      # [m]

    @property
    def n(self) -> int:
        return int(self.rod.shape[0])


def walls(x, dir_, length, diam, eta, dt, cutoff, wall_list, F=None) -> WallContacts:
    xa, d = _f64(x), _f64(dir_)
    n = xa.shape[0]
    la, l0 = _len_args(length, n)
    W = _f64(np.asarray(wall_list, dtype=np.float64).reshape(-1, 8))
    nw = W.shape[0]
    Fa = None if F is None else _f64(F)
    cap = 2 * n * max(nw, 1) + 1
    rod = np.empty(cap, np.int32)
    e, arm, phi, q = np.empty((cap, 3)), np.empty((cap, 2)), np.empty(cap), np.empty(cap)
    m = _load().ora_walls(n, _p(xa), _p(d), _p(la), l0, diam, eta, dt, cutoff, nw, _p(W), _p(Fa), cap, _p(rod),
                          _p(e), _p(arm), _p(phi), _p(q))
    return WallContacts(rod[:m].copy(), e[:m].copy(), arm[:m].copy(), phi[:m].copy(), q[:m].copy())


def general_all(pr=None, cs=None, lk=None, lg=None, wc: Optional[WallContacts] = None) -> General:
    """Contacts, then links, then wall contacts (kind 0, no Q side)."""
    g = general(pr, cs, lk, lg)
    if wc is None or wc.n == 0:
        return g
    m = wc.n
    return General(_i32(np.concatenate([g.pi, wc.rod])), _i32(np.concatenate([g.pj, -np.ones(m, np.int32)])),
                   _f64(np.concatenate([g.e, wc.e])), _f64(np.concatenate([g.arm, wc.arm])),
                   _f64(np.concatenate([g.q, wc.q])),
                   np.ascontiguousarray(np.concatenate([g.kind, np.zeros(m, np.uint8)]), dtype=np.uint8),
                   _f64(np.concatenate([g.cmp, np.zeros(m)])))


# --- Brownian force and stress ----------------------------------------------------

KT_300K = 1.380649e-23 * 300.0 * 1e18   # pN um (Boltzmann constant x 300 K)


def mobility_pow_block(d, L: float, diam: float, eta: float, power: float) -> np.ndarray:
    M = np.empty(36)
    _load().ora_mobility_pow_block(_p(_f64(d)), L, diam, eta, power, _p(M))
    return M.reshape(6, 6)


def brownian_force(dir_, length, diam, eta, dt, kT, xi) -> np.ndarray:
    """F_B = sqrt(2 kT / h) M^(-1/2) xi per rod (xi: [n, 6] standard normal draws)."""
    d = _f64(dir_)
    n = d.shape[0]
    la, l0 = _len_args(length, n)
    FB = np.empty((n, 6))
    _load().ora_brownian_force(n, _p(d), _p(la), l0, diam, eta, dt, kT, _p(_f64(xi)), _p(FB))
    return FB


def stress(x, dir_, length, box, pr: Pairs, cs: Constraints, gamma_pairs, lk: Optional[Links] = None,
           lg: Optional[LinkGeometry] = None, gamma_links=None):
    """Virial stress of the constraint forces between rods, (collision, link),
    each 3x3: sigma = (1/V) sum_c gamma_c (x_P - x_Q') (outer) e_c over the
    pairs (x_Q' the imaged centre) and over the links between two rods
    (x_P - x_Q' = r - s_P d_P + s_Q d_Q with r = length e the link vector;
    links to fixed points and walls are external), V the box volume.
    Positive trace for repulsion; the paper's pressure is Tr(sigma) / 3."""
    b = _box3(box)
    V = float(np.prod(b))
    x = _f64(x)
    d = _f64(dir_)
    sc = np.zeros((3, 3))
    if pr.n:
        shift = img_unpack(pr.img) * b
        rc = x[pr.pi] - (x[pr.pj] + shift)
        sc = np.einsum("c,ca,cb->ab", _f64(gamma_pairs), rc, cs.e) / V
    sl = np.zeros((3, 3))
    if lk is not None and lk.n:
        two = lk.q >= 0          # links to fixed points are external, like walls
        r = lg.length[two, None] * lg.e[two]
        rc = r - lk.arm[two, :1] * d[lk.p[two]] + lk.arm[two, 1:2] * d[lk.q[two]]
        sl = np.einsum("c,ca,cb->ab", _f64(gamma_links)[two], rc, lg.e[two]) / V
    return sc, sl


# --- crosslinker kinetics (kinetic Monte Carlo) ----------------------------------

AVOGADRO_UM3_PER_UM = 602.214076  # molecules per um^3 in a 1 uM solution
KMC_U, KMC_SA, KMC_SB, KMC_D = 0, 1, 2, 3
EV_NONE, EV_BIND, EV_UNBIND, EV_CROSS, EV_RELEASE = 0, 1, 2, 3, 4


class KmcParams(C.Structure):
    """Parameters of the crosslinker kinetics (units um, s, pN).  Association
    constants are volumes (um^3): a constant K in (uM)^-1 is
    K / AVOGADRO_UM3_PER_UM."""
    _fields_ = [("eps", C.c_double), ("Ka", C.c_double * 2), ("koS", C.c_double * 2), ("Ke", C.c_double * 2),
                ("koD", C.c_double * 2), ("kappa", C.c_double), ("rest", C.c_double), ("lam", C.c_double),
                ("xc", C.c_double), ("kT", C.c_double), ("rcs", C.c_double), ("rcd", C.c_double),
                ("dU", C.c_double), ("diam", C.c_double), ("dt", C.c_double)]


def kmc_params(*, eps, Ka, koS, Ke, koD, kappa, rest, lam, kT, rcs, rcd, dU, diam, dt, xc=0.0) -> KmcParams:
    pair = lambda v: (C.c_double * 2)(*((v, v) if np.isscalar(v) else v))  # noqa: E731
    return KmcParams(float(eps), pair(Ka), pair(koS), pair(Ke), pair(koD), float(kappa), float(rest), float(lam),
                     float(xc), float(kT), float(rcs), float(rcd), float(dU), float(diam), float(dt))


def kmc_effective_volume(P: KmcParams) -> float:
    return float(_load().ora_kmc_effective_volume(C.byref(P)))


def kmc_inside_length(x, dir_, length, box, i, point, r) -> float:
    x, d = _f64(x), _f64(dir_)
    la, l0 = _len_args(length, x.shape[0])
    return float(_load().ora_kmc_inside_length(x.shape[0], _p(x), _p(d), _p(la), l0, _p(_box3(box)), int(i),
                                               _p(_f64(point)), float(r)))


def kmc_cross_sum(x, dir_, length, box, P: KmcParams, point, skip=-1) -> float:
    x, d = _f64(x), _f64(dir_)
    la, l0 = _len_args(length, x.shape[0])
    return float(_load().ora_kmc_cross_sum(x.shape[0], _p(x), _p(d), _p(la), l0, _p(_box3(box)), C.byref(P),
                                           _p(_f64(point)), int(skip)))


@dataclass
class Crosslinkers:
    """state[m] (KMC_*), rod[m][2] and arc[m][2] (filament and arclength of
    heads A and B, -1 when unbound), x[m][3] (position: the crosslinker's when
    unbound, else the bound head's, head A's when both are bound)."""
    state: np.ndarray
    rod: np.ndarray
    arc: np.ndarray
    x: np.ndarray

    def copy(self) -> "Crosslinkers":
        return Crosslinkers(self.state.copy(), self.rod.copy(), self.arc.copy(), self.x.copy())


def kmc_step(x, dir_, length, box, P: KmcParams, Vbd: float, xl: Crosslinkers, u, xi) -> np.ndarray:
    """One step of the crosslinker kinetics, in place on xl; returns the
    event of each crosslinker (EV_*)."""
    x, d = _f64(x), _f64(dir_)
    la, l0 = _len_args(length, x.shape[0])
    m = xl.state.shape[0]
    for a, dt in ((xl.state, np.int32), (xl.rod, np.int32), (xl.arc, np.float64), (xl.x, np.float64)):
        assert a.dtype == dt and a.flags.c_contiguous
    u, xi = _f64(u), _f64(xi)
    assert u.shape == (m, 4) and xi.shape == (m, 3)
    ev = np.zeros(m, np.int32)
    _load().ora_kmc_step(x.shape[0], _p(x), _p(d), _p(la), l0, _p(_box3(box)), C.byref(P), float(Vbd), m,
                         _p(xl.state), _p(xl.rod), _p(xl.arc), _p(xl.x), _p(u), _p(xi), _p(ev))
    return ev
