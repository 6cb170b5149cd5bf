"""Python binding of librodlcp, the gfx950 HIP library for the steric-
constraint step of rigid filaments (Yan et al., arXiv 2109.08206).

Argument marshalling only: every step runs in the HIP kernels behind the
C-ABI declared in ``include/rodlcp.h``.  Tensors must be CUDA (HIP) tensors,
contiguous, float64 (int32 / uint8 for index and flag lists).  Work goes on
``torch.cuda.current_stream()``.  There is no CPU fallback: without the built
library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librodlcp.so")

OK, NOT_CONVERGED, STAGNATED = 0, 1, 2
ERR_ARG, ERR_CAPACITY, ERR_NONFINITE, ERR_HIP, ERR_NOMEM = -1, -2, -3, -4, -5
FP64, FP32_MIXED = 0, 1
TAPE_NONE, TAPE_RECORD, TAPE_REPLAY = 0, 1, 2
IMG_ZERO = 0x888

_lib = None
_lock = threading.Lock()


class RodLCPError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("diam", C.c_double), ("cutoff", C.c_double), ("eta", C.c_double),
                ("dt", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int64), ("precision", C.c_int32),
                ("check_every", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("residual", C.c_double), ("alpha0", C.c_double),
                ("status", C.c_int32), ("fp64_refreshes", C.c_int32)]


class RLLinks(C.Structure):
    _fields_ = [("n_links", C.c_int64), ("p", C.c_void_p), ("q", C.c_void_p), ("arm", C.c_void_p),
                ("kappa", C.c_void_p), ("rest", C.c_void_p), ("anchor", C.c_void_p), ("key", C.c_void_p)]


class RLWall(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p", C.c_double * 3), ("a", C.c_double * 3), ("r", C.c_double)]


WALL_PLANE, WALL_SPHERE_IN, WALL_CYLINDER_IN = 0, 1, 2


def walls_array(walls):
    """[(kind, p, a, r), ...] as an rl_wall array (host)."""
    arr = (RLWall * max(len(walls), 1))()
    for k, (kind, pt, ax, r) in enumerate(walls):
        arr[k].kind = int(kind)
        arr[k].p[:] = [float(v) for v in pt]
        arr[k].a[:] = [float(v) for v in ax]
        arr[k].r = float(r)
    return arr


class StepExtra(C.Structure):
    _fields_ = [("x_unwrapped", C.c_void_p), ("links", C.c_void_p), ("gamma_links", C.c_void_p),
                ("n_walls", C.c_int32), ("walls", C.c_void_p), ("n_wall_contacts", C.c_void_p),
                ("noise", C.c_void_p), ("kT", C.c_double), ("warm_start", C.c_int32), ("stress", C.c_void_p)]


class KmcParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("Ka", C.c_double * 2), ("koS", C.c_double * 2), ("Ke", C.c_double * 2),
                ("koD", C.c_double * 2), ("kappa", C.c_double), ("rest", C.c_double), ("lam", C.c_double),
                ("xc", C.c_double), ("kT", C.c_double), ("rcs", C.c_double), ("rcd", C.c_double),
                ("dU", C.c_double)]


def kmc_params(*, eps, Ka, koS, Ke, koD, kappa, rest, lam, kT, rcs, rcd, dU, xc=0.0) -> KmcParams:
    """rl_kmc_params; Ka, koS, Ke, koD a number (both heads) or a pair (A, B).
    Association constants in um^3."""
    pair = lambda v: (C.c_double * 2)(*((float(v), float(v)) if isinstance(v, (int, float)) else  # noqa: E731
                                       (float(v[0]), float(v[1]))))
    return KmcParams(float(eps), pair(Ka), pair(koS), pair(Ke), pair(koD), float(kappa), float(rest), float(lam),
                     float(xc), float(kT), float(rcs), float(rcd), float(dU))


class RLCrosslinkers(C.Structure):
    _fields_ = [("m", C.c_int64), ("state", C.c_void_p), ("rod", C.c_void_p), ("arc", C.c_void_p),
                ("x", C.c_void_p)]


XL_U, XL_SA, XL_SB, XL_D = 0, 1, 2, 3
EV_NONE, EV_BIND, EV_UNBIND, EV_CROSS, EV_RELEASE = 0, 1, 2, 3, 4


class AdjointInfo(C.Structure):
    _fields_ = [("cg_iterations", C.c_int64), ("cg_residual", C.c_double), ("n_active", C.c_int64),
                ("status", C.c_int32), ("solve_status", C.c_int32), ("solve_iterations", C.c_int64),
                ("solve_residual", C.c_double)]


SYMBOLS = ("rl_create", "rl_destroy", "rl_set_params", "rl_get_params", "rl_set_stream", "rl_reserve",
           "rl_status_str", "rl_last_error", "rl_directors", "rl_build_pairs", "rl_assemble_D", "rl_apply_M",
           "rl_solve_lcp", "rl_step", "rl_profile_enable", "rl_profile_read", "rl_solve_lcp_batched",
           "rl_batch_tuning", "rl_solve_lcp_adjoint", "rl_step_adjoint", "rl_solve_lcp_noalloc",
           "rl_assemble_links", "rl_solve_general", "rl_assemble_walls", "rl_kmc_effective_volume", "rl_kmc_step",
           "rl_kmc_links")


def load(path: Optional[str] = None) -> C.CDLL:
    """Load the built library (never builds, never falls back)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(f"librodlcp.so not built ({p}); run paper_2109_08206_amd/build.py")
        lib = C.CDLL(p)
        P, I64, D, I32 = C.c_void_p, C.c_int64, C.c_double, C.c_int32
        H = C.c_void_p
        sig = {
            "rl_create": ([C.POINTER(H), C.POINTER(Params)], C.c_int),
            "rl_destroy": ([H], C.c_int),
            "rl_set_params": ([H, C.POINTER(Params)], C.c_int),
            "rl_get_params": ([H, C.POINTER(Params)], C.c_int),
            "rl_set_stream": ([H, P], C.c_int),
            "rl_reserve": ([H, I64, I64], C.c_int),
            "rl_status_str": ([C.c_int], C.c_char_p),
            "rl_last_error": ([], C.c_char_p),
            "rl_directors": ([H, I64, P, P], C.c_int),
            "rl_build_pairs": ([H, I64, P, P, P, D, I64, P, P, P, P, C.POINTER(C.c_int64)], C.c_int),
            "rl_assemble_D": ([H, I64, P, P, P, D, I64, P, P, P, P, P, P, P, P], C.c_int),
            "rl_apply_M": ([H, I64, P, P, D, I64, P, P, P, P, P, P, P], C.c_int),
            "rl_solve_lcp": ([H, I64, P, P, D, I64, P, P, P, P, P, P, P, P, C.POINTER(SolveInfo)], C.c_int),
            "rl_solve_lcp_noalloc": ([H, I64, P, P, D, I64, P, P, P, P, P, P, P, P, C.POINTER(SolveInfo)],
                                     C.c_int),
            "rl_assemble_links": ([H, I64, P, P, P, D, C.POINTER(RLLinks), P, P, P, P, P, P], C.c_int),
            "rl_solve_general": ([H, I64, P, P, D, I64, P, P, P, P, P, P, P, P, P, P, C.POINTER(SolveInfo)],
                                 C.c_int),
            "rl_assemble_walls": ([H, I64, P, P, P, D, P, I32, P, I64, P, P, P, P, P, P, C.POINTER(C.c_int64)],
                                  C.c_int),
            "rl_step": ([H, I64, P, P, P, D, P, P, C.POINTER(SolveInfo), C.POINTER(C.c_int64), P, I64, I32,
                         C.POINTER(StepExtra)], C.c_int),
            "rl_profile_enable": ([H, C.c_int], C.c_int),
            "rl_solve_lcp_batched": ([H, I32, P, P, P, P, D, P, P, P, P, P, P, P, P, P], C.c_int),
            "rl_batch_tuning": ([H, C.c_int, C.c_int, P], C.c_int),
            "rl_profile_read": ([H, C.POINTER(C.c_double)], C.c_int),
            "rl_solve_lcp_adjoint": ([H, I64, P, P, D, I64, P, P, P, P, P, P, P, P, D, P, P, P, P, P,
                                      C.POINTER(AdjointInfo)], C.c_int),
            "rl_step_adjoint": ([H, I64, P, P, P, D, P, P, I64, P, P, P, D, C.POINTER(AdjointInfo)], C.c_int),
            "rl_kmc_effective_volume": ([H, C.POINTER(KmcParams), C.POINTER(C.c_double)], C.c_int),
            "rl_kmc_step": ([H, I64, P, P, P, D, C.POINTER(KmcParams), C.POINTER(RLCrosslinkers), P, P, P,
                             C.POINTER(C.c_int64)], C.c_int),
            "rl_kmc_links": ([H, C.POINTER(KmcParams), C.POINTER(RLCrosslinkers), I64, P, P, P, P, P, P,
                              C.POINTER(C.c_int64)], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def _torch():
    import torch
    return torch


def _ptr(t, dtype=None, shape=None, name="array"):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name}: expected a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _len_args(length, n):
    """(len tensor or None, uniform length)."""
    torch = _torch()
    if isinstance(length, torch.Tensor):
        return _ptr(length, torch.float64, (n,), "len"), 0.0
    return None, float(length)


@dataclass
class SolveResult:
    iterations: int
    residual: float
    alpha0: float
    status: int
    fp64_refreshes: int = 0


@dataclass
class AdjointResult:
    cg_iterations: int
    cg_residual: float
    n_active: int
    status: int
    solve_status: int
    solve_iterations: int
    solve_residual: float


def _adj_result(info) -> "AdjointResult":
    return AdjointResult(int(info.cg_iterations), float(info.cg_residual), int(info.n_active), int(info.status),
                         int(info.solve_status), int(info.solve_iterations), float(info.solve_residual))


def _result(info) -> "SolveResult":
    return SolveResult(int(info.iterations), float(info.residual), float(info.alpha0), int(info.status),
                       int(info.fp64_refreshes))


class Solver:
    """One library handle: parameters, stream and workspace."""

    def __init__(self, box, diam=0.025, cutoff=0.05, eta=0.01, dt=1e-4, tol=1e-8, max_iter=100_000,
                 precision=FP64, check_every=0):
        self.lib = load()
        self._h = C.c_void_p()
        self.params = Params()
        self.set_params(box=box, diam=diam, cutoff=cutoff, eta=eta, dt=dt, tol=tol, max_iter=max_iter,
                        precision=precision, check_every=check_every, _create=True)

    # -- lifecycle ------------------------------------------------------------
    def set_params(self, _create=False, **kw):
        p = self.params
        box = kw.pop("box", None)
        if box is not None:
            b = [float(box)] * 3 if not hasattr(box, "__len__") else [float(v) for v in box]
            p.box[:] = b
        for k, v in kw.items():
            setattr(p, k, v)
        if _create:
            self._check(self.lib.rl_create(C.byref(self._h), C.byref(p)), "rl_create")
        else:
            self._check(self.lib.rl_set_params(self._h, C.byref(p)), "rl_set_params")

    def close(self):
        if self._h:
            self.lib.rl_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, where):
        if rc < 0:
            raise RodLCPError(rc, where, self.lib.rl_last_error().decode())
        return rc

    def _stream(self):
        torch = _torch()
        self.lib.rl_set_stream(self._h, C.c_void_p(torch.cuda.current_stream().cuda_stream))

    def profile_enable(self, every: int):
        self._check(self.lib.rl_profile_enable(self._h, int(every)), "rl_profile_enable")

    def profile_read(self):
        """{'rod_ms', 'rod_launches', 'con_ms', 'con_launches'} since the last read."""
        out = (C.c_double * 4)()
        self._check(self.lib.rl_profile_read(self._h, out), "rl_profile_read")
        return {"rod_ms": out[0], "rod_launches": int(out[1]), "con_ms": out[2], "con_launches": int(out[3])}

    def reserve(self, max_rods, max_pairs):
        self._check(self.lib.rl_reserve(self._h, int(max_rods), int(max_pairs)), "rl_reserve")

    # -- entry points -----------------------------------------------------------
    def directors(self, quat, out=None):
        torch = _torch()
        n = quat.shape[0]
        out = torch.empty((n, 3), dtype=torch.float64, device=quat.device) if out is None else out
        self._stream()
        self._check(self.lib.rl_directors(self._h, n, _ptr(quat, torch.float64, (n, 4), "quat"),
                                          _ptr(out, torch.float64, (n, 3), "dir")), "rl_directors")
        return out

    def build_pairs(self, x, dir_, length, capacity=None):
        """Returns (pi, pj, img, flags), each trimmed to the pair count."""
        torch = _torch()
        n = x.shape[0]
        la, l0 = _len_args(length, n)
        cap = int(capacity) if capacity is not None else 16 * n + 64
        for _ in range(2):
            dev = x.device
            pi = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            pj = torch.empty_like(pi)
            img = torch.empty_like(pi)
            fl = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
            cnt = C.c_int64(0)
            self._stream()
            rc = self.lib.rl_build_pairs(self._h, n, _ptr(x, torch.float64, (n, 3), "x"),
                                         _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, cap,
                                         _ptr(pi), _ptr(pj), _ptr(img), _ptr(fl), C.byref(cnt))
            if rc == ERR_CAPACITY and capacity is None:
                cap = int(cnt.value)
                continue
            self._check(rc, "rl_build_pairs")
            k = int(cnt.value)
            return pi[:k], pj[:k], img[:k], fl[:k]
        raise RodLCPError(ERR_CAPACITY, "rl_build_pairs", "capacity")

    def assemble_D(self, x, dir_, length, pi, pj, img, F):
        torch = _torch()
        n, nc = x.shape[0], pi.shape[0]
        la, l0 = _len_args(length, n)
        dev = x.device
        phi = torch.empty(nc, dtype=torch.float64, device=dev)
        e = torch.empty((nc, 3), dtype=torch.float64, device=dev)
        arm = torch.empty((nc, 2), dtype=torch.float64, device=dev)
        q = torch.empty(nc, dtype=torch.float64, device=dev)
        self._stream()
        self._check(self.lib.rl_assemble_D(
            self._h, n, _ptr(x, torch.float64, (n, 3), "x"), _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, nc,
            _ptr(pi, torch.int32, (nc,), "pi"), _ptr(pj, torch.int32, (nc,), "pj"),
            _ptr(img, torch.int32, (nc,), "img"), _ptr(F, torch.float64, (n, 6), "F"),
            _ptr(phi), _ptr(e), _ptr(arm), _ptr(q)), "rl_assemble_D")
        return phi, e, arm, q

    def apply_M(self, dir_, length, pi, pj, e, arm, q, gamma, out=None):
        torch = _torch()
        n, nc = dir_.shape[0], pi.shape[0]
        la, l0 = _len_args(length, n)
        w = torch.empty(nc, dtype=torch.float64, device=dir_.device) if out is None else out
        self._stream()
        self._check(self.lib.rl_apply_M(
            self._h, n, _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, nc, _ptr(pi, torch.int32, (nc,), "pi"),
            _ptr(pj, torch.int32, (nc,), "pj"), _ptr(e, torch.float64, (nc, 3), "e"),
            _ptr(arm, torch.float64, (nc, 2), "arm"), _ptr(q, torch.float64, (nc,), "q"),
            _ptr(gamma, torch.float64, (nc,), "gamma"), _ptr(w, torch.float64, (nc,), "w")), "rl_apply_M")
        return w

    def solve_lcp(self, dir_, length, pi, pj, e, arm, q, F=None, gamma=None, U=None):
        """Returns (gamma, U, SolveResult); gamma is updated in place if given."""
        torch = _torch()
        n, nc = dir_.shape[0], pi.shape[0]
        la, l0 = _len_args(length, n)
        dev = dir_.device
        gamma = torch.zeros(nc, dtype=torch.float64, device=dev) if gamma is None else gamma
        U = torch.empty((n, 6), dtype=torch.float64, device=dev) if U is None else U
        info = SolveInfo()
        self._stream()
        rc = self.lib.rl_solve_lcp(
            self._h, n, _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, nc, _ptr(pi, torch.int32, (nc,), "pi"),
            _ptr(pj, torch.int32, (nc,), "pj"), _ptr(e, torch.float64, (nc, 3), "e"),
            _ptr(arm, torch.float64, (nc, 2), "arm"), _ptr(q, torch.float64, (nc,), "q"),
            _ptr(F, torch.float64, (n, 6), "F"), _ptr(gamma, torch.float64, (nc,), "gamma"),
            _ptr(U, torch.float64, (n, 6), "U"), C.byref(info))
        self._check(rc, "rl_solve_lcp")
        return gamma, U, _result(info)

    def solve_lcp_noalloc(self, dir_, length, pi, pj, e, arm, q, gamma, U, F=None):
        """solve_lcp without device allocation (workspace in the library's
        scratch array): gamma (start, updated in place) and U must be given."""
        torch = _torch()
        n, nc = dir_.shape[0], pi.shape[0]
        la, l0 = _len_args(length, n)
        info = SolveInfo()
        self._stream()
        rc = self.lib.rl_solve_lcp_noalloc(
            self._h, n, _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, nc, _ptr(pi, torch.int32, (nc,), "pi"),
            _ptr(pj, torch.int32, (nc,), "pj"), _ptr(e, torch.float64, (nc, 3), "e"),
            _ptr(arm, torch.float64, (nc, 2), "arm"), _ptr(q, torch.float64, (nc,), "q"),
            _ptr(F, torch.float64, (n, 6), "F"), _ptr(gamma, torch.float64, (nc,), "gamma"),
            _ptr(U, torch.float64, (n, 6), "U"), C.byref(info))
        self._check(rc, "rl_solve_lcp_noalloc")
        return gamma, U, _result(info)

    @staticmethod
    def links_struct(p, q, arm, kappa, rest, anchor=None, key=None):
        """An rl_links over device tensors (kept alive by the caller); key:
        optional int64 warm-start keys."""
        torch = _torch()
        nl = p.shape[0]
        return RLLinks(nl, _ptr(p, torch.int32, (nl,), "p"), _ptr(q, torch.int32, (nl,), "q"),
                       _ptr(arm, torch.float64, (nl, 2), "arm"), _ptr(kappa, torch.float64, (nl,), "kappa"),
                       _ptr(rest, torch.float64, (nl,), "rest"),
                       _ptr(anchor, torch.float64, (nl, 3), "anchor"), _ptr(key, torch.int64, (nl,), "key"))

    def assemble_links(self, x, dir_, length, p, q, arm, kappa, rest, anchor=None, F=None):
        """Link geometry: returns (length, e, q, cmp, flags)."""
        torch = _torch()
        n, nl = x.shape[0], p.shape[0]
        la, l0 = _len_args(length, n)
        dev = x.device
        L = torch.empty(nl, dtype=torch.float64, device=dev)
        e = torch.empty((nl, 3), dtype=torch.float64, device=dev)
        qq = torch.empty(nl, dtype=torch.float64, device=dev)
        cmp = torch.empty(nl, dtype=torch.float64, device=dev)
        fl = torch.empty(max(nl, 1), dtype=torch.uint8, device=dev)
        lk = self.links_struct(p, q, arm, kappa, rest, anchor)
        self._stream()
        self._check(self.lib.rl_assemble_links(self._h, n, _ptr(x, torch.float64, (n, 3), "x"),
                                               _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, C.byref(lk),
                                               _ptr(F, torch.float64, (n, 6), "F"), _ptr(L), _ptr(e), _ptr(qq),
                                               _ptr(cmp), _ptr(fl)), "rl_assemble_links")
        return L, e, qq, cmp, fl[:nl]

    def assemble_walls(self, x, dir_, length, walls, F=None, capacity=None):
        """Wall constraints of the rods: returns (rod, e, arm, phi, q, flags)."""
        torch = _torch()
        n = x.shape[0]
        la, l0 = _len_args(length, n)
        cap = int(capacity) if capacity is not None else 2 * n * max(len(walls), 1)
        dev = x.device
        rod = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        e = torch.empty((max(cap, 1), 3), dtype=torch.float64, device=dev)
        arm = torch.empty((max(cap, 1), 2), dtype=torch.float64, device=dev)
        phi = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        q = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        fl = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
        wl = walls_array(walls)
        cnt = C.c_int64(0)
        self._stream()
        self._check(self.lib.rl_assemble_walls(
            self._h, n, _ptr(x, torch.float64, (n, 3), "x"), _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0,
            _ptr(F, torch.float64, (n, 6), "F"), len(walls), C.cast(wl, C.c_void_p), cap, _ptr(rod), _ptr(e),
            _ptr(arm), _ptr(phi), _ptr(q), _ptr(fl), C.byref(cnt)), "rl_assemble_walls")
        m = int(cnt.value)
        return rod[:m], e[:m], arm[:m], phi[:m], q[:m], fl[:m]

    def kmc_effective_volume(self, kp: KmcParams) -> float:
        out = C.c_double(0.0)
        self._check(self.lib.rl_kmc_effective_volume(self._h, C.byref(kp), C.byref(out)), "rl_kmc_effective_volume")
        return float(out.value)

    @staticmethod
    def _xl_struct(state, rod, arc, x):
        torch = _torch()
        m = state.shape[0]
        return RLCrosslinkers(m, _ptr(state, torch.int32, (m,), "state"), _ptr(rod, torch.int32, (m, 2), "rod"),
                              _ptr(arc, torch.float64, (m, 2), "arc"), _ptr(x, torch.float64, (m, 3), "x"))

    def kmc_step(self, x, dir_, length, kp: KmcParams, state, rod, arc, xl, u, xi, event=None):
        """One step of the crosslinker kinetics; (state, rod, arc, xl) are
        updated in place.  Returns the counts of each event (5 ints)."""
        torch = _torch()
        n, m = x.shape[0], state.shape[0]
        la, l0 = _len_args(length, n)
        X = self._xl_struct(state, rod, arc, xl)
        counts = (C.c_int64 * 5)()
        self._stream()
        self._check(self.lib.rl_kmc_step(
            self._h, n, _ptr(x, torch.float64, (n, 3), "x"), _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0,
            C.byref(kp), C.byref(X), _ptr(u, torch.float64, (m, 4), "u"), _ptr(xi, torch.float64, (m, 3), "xi"),
            _ptr(event, torch.int32, (m,), "event"), counts), "rl_kmc_step")
        return [int(v) for v in counts]

    def kmc_links(self, kp: KmcParams, state, rod, arc, capacity=None, keys=False):
        """The doubly bound crosslinkers as links: (p, q, arm, kappa, rest),
        and with keys=True also their warm-start keys (the crosslinker
        indices)."""
        torch = _torch()
        m = state.shape[0]
        cap = int(capacity) if capacity is not None else m
        dev = state.device
        p = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        q = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        arm = torch.empty((max(cap, 1), 2), dtype=torch.float64, device=dev)
        kap = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        rest = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        key = torch.empty(max(cap, 1), dtype=torch.int64, device=dev) if keys else None
        X = RLCrosslinkers(m, _ptr(state, torch.int32, (m,), "state"), _ptr(rod, torch.int32, (m, 2), "rod"),
                           _ptr(arc, torch.float64, (m, 2), "arc"), None)
        cnt = C.c_int64(0)
        self._stream()
        self._check(self.lib.rl_kmc_links(self._h, C.byref(kp), C.byref(X), cap, _ptr(p), _ptr(q), _ptr(arm),
                                          _ptr(kap), _ptr(rest), _ptr(key), C.byref(cnt)), "rl_kmc_links")
        k = int(cnt.value)
        if keys:
            return p[:k], q[:k], arm[:k], kap[:k], rest[:k], key[:k]
        return p[:k], q[:k], arm[:k], kap[:k], rest[:k]

    def solve_general(self, dir_, length, pi, pj, e, arm, q, kind, cmp, F=None, gamma=None, U=None):
        """Mixed unilateral/bilateral problem over a general list (any order;
        pj = -1 for a fixed body).  Returns (gamma, U, SolveResult)."""
        torch = _torch()
        n, nc = dir_.shape[0], pi.shape[0]
        la, l0 = _len_args(length, n)
        dev = dir_.device
        gamma = torch.zeros(nc, dtype=torch.float64, device=dev) if gamma is None else gamma
        U = torch.empty((n, 6), dtype=torch.float64, device=dev) if U is None else U
        info = SolveInfo()
        self._stream()
        rc = self.lib.rl_solve_general(
            self._h, n, _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, nc, _ptr(pi, torch.int32, (nc,), "pi"),
            _ptr(pj, torch.int32, (nc,), "pj"), _ptr(e, torch.float64, (nc, 3), "e"),
            _ptr(arm, torch.float64, (nc, 2), "arm"), _ptr(q, torch.float64, (nc,), "q"),
            _ptr(kind, torch.uint8, (nc,), "kind"), _ptr(cmp, torch.float64, (nc,), "cmp"),
            _ptr(F, torch.float64, (n, 6), "F"), _ptr(gamma, torch.float64, (nc,), "gamma"),
            _ptr(U, torch.float64, (n, 6), "U"), C.byref(info))
        self._check(rc, "rl_solve_general")
        return gamma, U, _result(info)

    def solve_lcp_batched(self, rod_off, pair_off, dir_, length, pi, pj, e, arm, q, F=None, gamma=None, U=None):
        """S systems concatenated (rod_off, pair_off: S+1 host offsets; pi, pj
        index the concatenated rods).  Returns (gamma, U, [SolveResult] * S)."""
        import numpy as np
        torch = _torch()
        ro = np.ascontiguousarray(rod_off, dtype=np.int64)
        po = np.ascontiguousarray(pair_off, dtype=np.int64)
        S = ro.shape[0] - 1
        n, nc = int(ro[-1]), int(po[-1])
        la, l0 = _len_args(length, n)
        dev = dir_.device
        gamma = torch.zeros(nc, dtype=torch.float64, device=dev) if gamma is None else gamma
        U = torch.empty((n, 6), dtype=torch.float64, device=dev) if U is None else U
        infos = (SolveInfo * S)()
        self._stream()
        rc = self.lib.rl_solve_lcp_batched(
            self._h, S, ro.ctypes.data_as(C.c_void_p), po.ctypes.data_as(C.c_void_p),
            _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, _ptr(pi, torch.int32, (nc,), "pi"),
            _ptr(pj, torch.int32, (nc,), "pj"), _ptr(e, torch.float64, (nc, 3), "e"),
            _ptr(arm, torch.float64, (nc, 2), "arm"), _ptr(q, torch.float64, (nc,), "q"),
            _ptr(F, torch.float64, (n, 6), "F"), _ptr(gamma, torch.float64, (nc,), "gamma"),
            _ptr(U, torch.float64, (n, 6), "U"), infos)
        self._check(rc, "rl_solve_lcp_batched")
        return gamma, U, [_result(i) for i in infos]

    def batch_tuning(self, rod_block: int = 0, con_block: int = 0):
        """Fix the batched workgroup sizes (0, 0 = time them); returns the
        sizes the last batched solve used."""
        out = (C.c_int * 2)()
        self._check(self.lib.rl_batch_tuning(self._h, int(rod_block), int(con_block), out), "rl_batch_tuning")
        return int(out[0]), int(out[1])

    def step(self, x, quat, length, F=None, U=None, tape=None, tape_mode=TAPE_NONE, x_unwrapped=None,
             links=None, gamma_links=None, walls=None, noise=None, kT=0.0, warm_start=False, stress=False):
        """One whole timestep in place on x and quat; returns (U, SolveResult, n_pairs).
        tape: float64 device tensor for the step's constraint forces
        (TAPE_RECORD writes them, TAPE_REPLAY starts from them).
        x_unwrapped: [n, 3] centres without wrapping, advanced in place.
        links: (p, q, arm, kappa, rest, anchor[, key]) device tensors (anchor may be
        None; key: warm-start keys), solved with the contacts; gamma_links
        receives their forces.
        walls: [(kind, p, a, r), ...].  The step's wall constraint count is
        left in self.last_wall_contacts.
        noise: [n, 6] N(0,1) draws with kT > 0: Brownian force.
        warm_start: start from the last warm step's forces (and keep these).
        stress: leave the contact and link virial stresses (2 x 3 x 3, numpy)
        in self.last_stress."""
        torch = _torch()
        n = x.shape[0]
        la, l0 = _len_args(length, n)
        U = torch.empty((n, 6), dtype=torch.float64, device=x.device) if U is None else U
        info = SolveInfo()
        npairs = C.c_int64(0)
        tlen = 0 if tape is None else int(tape.shape[0])
        lk = self.links_struct(*links) if links is not None else None
        wl = walls_array(walls) if walls else None
        nwc = C.c_int64(0)
        nl = 0 if links is None else int(links[0].shape[0])
        sbuf = (C.c_double * 18)() if stress else None
        extra = StepExtra(_ptr(x_unwrapped, torch.float64, (n, 3), "x_unwrapped"),
                          C.cast(C.pointer(lk), C.c_void_p) if lk is not None else None,
                          _ptr(gamma_links, torch.float64, (nl,), "gamma_links"), len(walls) if walls else 0,
                          C.cast(wl, C.c_void_p) if wl is not None else None,
                          C.cast(C.pointer(nwc), C.c_void_p), _ptr(noise, torch.float64, (n, 6), "noise"),
                          float(kT), 1 if warm_start else 0, C.cast(sbuf, C.c_void_p) if stress else None)
        self._stream()
        rc = self.lib.rl_step(self._h, n, _ptr(x, torch.float64, (n, 3), "x"),
                              _ptr(quat, torch.float64, (n, 4), "quat"), la, l0,
                              _ptr(F, torch.float64, (n, 6), "F"), _ptr(U, torch.float64, (n, 6), "U"),
                              C.byref(info), C.byref(npairs), _ptr(tape, torch.float64, None, "tape"), tlen,
                              int(tape_mode), C.byref(extra))
        self.last_wall_contacts = int(nwc.value)
        if stress:
            import numpy as np
            self.last_stress = np.array(list(sbuf)).reshape(2, 3, 3)
        if rc == ERR_CAPACITY and tape_mode == TAPE_RECORD:
            err = RodLCPError(rc, "rl_step", f"tape too short for {int(npairs.value)} constraints")
            err.count = int(npairs.value)
            raise err
        self._check(rc, "rl_step")
        return U, _result(info), int(npairs.value)

    def step_recording(self, x, quat, length, F=None, U=None, capacity=None, x_unwrapped=None):
        """step() that records its tape; returns (U, SolveResult, tape)."""
        torch = _torch()
        cap = int(capacity) if capacity is not None else 16 * x.shape[0] + 64
        for _ in range(2):
            tape = torch.empty(max(cap, 1), dtype=torch.float64, device=x.device)
            try:
                U, info, npairs = self.step(x, quat, length, F=F, U=U, tape=tape, tape_mode=TAPE_RECORD,
                                            x_unwrapped=x_unwrapped)
                return U, info, tape[:npairs]
            except RodLCPError as err:
                if err.status != ERR_CAPACITY:
                    raise
                cap = err.count
        raise RodLCPError(ERR_CAPACITY, "rl_step", "tape capacity")

    def solve_lcp_adjoint(self, dir_, length, pi, pj, e, arm, q, gamma, U_bar, F=None, cg_tol=0.0):
        """Adjoint of solve_lcp as the map (dir, e, arm, q, F) -> U at its
        solution gamma.  Returns (q_bar, e_bar, arm_bar, F_bar, dir_bar,
        AdjointResult)."""
        torch = _torch()
        n, nc = dir_.shape[0], pi.shape[0]
        la, l0 = _len_args(length, n)
        dev = dir_.device
        qb = torch.empty(nc, dtype=torch.float64, device=dev)
        eb = torch.empty((nc, 3), dtype=torch.float64, device=dev)
        ab = torch.empty((nc, 2), dtype=torch.float64, device=dev)
        Fb = torch.empty((n, 6), dtype=torch.float64, device=dev)
        db = torch.empty((n, 3), dtype=torch.float64, device=dev)
        info = AdjointInfo()
        self._stream()
        rc = self.lib.rl_solve_lcp_adjoint(
            self._h, n, _ptr(dir_, torch.float64, (n, 3), "dir"), la, l0, nc, _ptr(pi, torch.int32, (nc,), "pi"),
            _ptr(pj, torch.int32, (nc,), "pj"), _ptr(e, torch.float64, (nc, 3), "e"),
            _ptr(arm, torch.float64, (nc, 2), "arm"), _ptr(q, torch.float64, (nc,), "q"),
            _ptr(F, torch.float64, (n, 6), "F"), _ptr(gamma, torch.float64, (nc,), "gamma"),
            _ptr(U_bar, torch.float64, (n, 6), "U_bar"), float(cg_tol), _ptr(qb), _ptr(eb), _ptr(ab), _ptr(Fb),
            _ptr(db), C.byref(info))
        self._check(rc, "rl_solve_lcp_adjoint")
        return qb, eb, ab, Fb, db, _adj_result(info)

    def step_adjoint(self, x, quat, length, F, x_bar, quat_bar, F_bar=None, cg_tol=0.0, tape=None):
        """Adjoint of step() at (x, quat, F): x_bar and quat_bar hold the
        adjoints of the step's outputs on entry and of its inputs on return
        (in place).  tape: the step's recorded constraint forces (optional).
        Returns (F_bar, AdjointResult)."""
        torch = _torch()
        n = x.shape[0]
        la, l0 = _len_args(length, n)
        F_bar = torch.empty((n, 6), dtype=torch.float64, device=x.device) if F_bar is None else F_bar
        info = AdjointInfo()
        tlen = 0 if tape is None else int(tape.shape[0])
        self._stream()
        rc = self.lib.rl_step_adjoint(
            self._h, n, _ptr(x, torch.float64, (n, 3), "x"), _ptr(quat, torch.float64, (n, 4), "quat"), la, l0,
            _ptr(F, torch.float64, (n, 6), "F"), _ptr(tape, torch.float64, None, "tape"), tlen,
            _ptr(x_bar, torch.float64, (n, 3), "x_bar"),
            _ptr(quat_bar, torch.float64, (n, 4), "quat_bar"), _ptr(F_bar, torch.float64, (n, 6), "F_bar"),
            float(cg_tol), C.byref(info))
        self._check(rc, "rl_step_adjoint")
        return F_bar, _adj_result(info)


def status_str(status: int) -> str:
    return load().rl_status_str(int(status)).decode()
