"""Gradients of the steric step and of a rollout, for checking the adjoint.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module; the product library never does.  It
shares no code with the HIP library.

Where the step is differentiable, the problem is an equality system on the
set A of active constraints.  The constraint rows in A hold as equalities
w_A = Mc_AA gamma_A + q_A = 0 (eq. linearconstraints; the complementarity
conditions of eq. cqpdef with gamma_A > 0), and the others have gamma = 0.
So, with A and the pair list held fixed, gamma_A = -Mc_AA^{-1} q_A and
U = M (D_A gamma_A + F) are smooth functions of the configuration and the
forces.  This module writes that map out densely in PyTorch (float64, CPU):
  * the director R(theta) z of the rotation of Section "rigid body kinematics";
  * the clamped closest points of the two axes (the oracle's own rule);
  * the slender-body mobility blocks;
  * the columns of D (eq. blockdef);
  * q = Phi/h + D^T M F;
  * gamma_A, U, and the Euler update of x and theta (eq. linearized Euler).
Reverse-mode automatic differentiation of it gives the oracle gradient.  A
is taken from the oracle's own BBPGD solve: c is in A when gamma_c > w_c
(the larger of the complementary pair is the one that is not zero).

Readings taken where the step is not differentiable:
  * Pairs whose axes are parallel (1 - (di.dj)^2 <= 1e-14) take the closest
    points from the midpoint rule.  Those points are held fixed; their
    derivative is not taken.  Likewise the contact normal of intersecting
    axes (distance < 1e-12).
  * Periodic wrapping shifts a centre by whole box lengths.  Its
    derivative is the identity.
  * theta_bar is reported on the unit sphere: its component along theta is
    removed (the step renormalises theta, so that component has no effect).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import (apply_Mc, assemble, bbpgd, closest, directors, img_unpack, integrate, mobility_coeffs, pairs,
               velocity, Pairs, Constraints)

EPS_PAR = 1e-14      # parallel axes (the oracle's closest-point rule)
DEGEN_DIST = 1e-12   # intersecting axes

_T = torch.float64


def _t(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


# --- pieces of the step, differentiable -------------------------------------

def directors_t(quat: torch.Tensor) -> torch.Tensor:
    """Body axis z carried by the rotation of theta = (s, p):
    R z = (s^2 - p.p) z + 2 p_z p + 2 s (p x z)."""
    s, p = quat[:, 0], quat[:, 1:]
    ez = torch.zeros_like(p)
    ez[:, 2] = 1.0
    return ((s * s - (p * p).sum(1))[:, None] * ez + 2.0 * p[:, 2:3] * p
            + 2.0 * s[:, None] * torch.linalg.cross(p, ez, dim=1))


def mobility_t(dir_: torch.Tensor, lengths: np.ndarray, diam: float, eta: float):
    """Per-rod 3x3 translational and rotational mobility blocks:
    a_perp I + (a_par - a_perp) d d^T and r_perp I + (r_par - r_perp) d d^T."""
    n = dir_.shape[0]
    co = np.array([mobility_coeffs(float(L), diam, eta) for L in lengths]) if n else np.zeros((0, 4))
    co = _t(co)
    I = torch.eye(3, dtype=_T).expand(n, 3, 3)
    ddt = dir_[:, :, None] * dir_[:, None, :]
    Mt = co[:, 1, None, None] * I + (co[:, 0] - co[:, 1])[:, None, None] * ddt
    Mr = co[:, 2, None, None] * I + (co[:, 3] - co[:, 2])[:, None, None] * ddt
    return Mt, Mr


def apply_M_t(Mt, Mr, G: torch.Tensor) -> torch.Tensor:
    """U = M G per rod, G [n, 6]."""
    ut = torch.einsum("nab,nb->na", Mt, G[:, :3])
    ur = torch.einsum("nab,nb->na", Mr, G[:, 3:])
    return torch.cat([ut, ur], 1)


@dataclass
class Fixed:
    """What is held fixed while differentiating one step."""
    pi: np.ndarray          # [nc]
    pj: np.ndarray          # [nc]
    shift: np.ndarray       # [nc, 3] periodic shift of rod j (box units times box)
    active: np.ndarray      # [nc] bool
    par_st: dict            # c -> (s, t) for parallel pairs
    degen_e: dict           # c -> e for intersecting axes


def closest_t(xi, di, hi, xj, dj, hj, fixed: Fixed):
    """Closest points of the two axes by the clamped normal equations
    (Lumelsky 1985; Ericson 2005, 5.1.9), the same rule as the oracle's C
    code, written with differentiable operations."""
    r0 = xi - xj
    b = (di * dj).sum(1)
    c = (di * r0).sum(1)
    f = (dj * r0).sum(1)
    den = 1.0 - b * b
    par = (den <= EPS_PAR).detach()
    den_s = torch.where(par, torch.ones_like(den), den)
    s1 = torch.minimum(torch.maximum((b * f - c) / den_s, -hi), hi)
    t1 = b * s1 + f
    tc = torch.minimum(torch.maximum(t1, -hj), hj)
    s2 = torch.minimum(torch.maximum(b * tc - c, -hi), hi)
    out = ((t1 < -hj) | (t1 > hj)).detach()
    s = torch.where(out, s2, s1)
    t = tc
    if fixed.par_st:
        idx = torch.tensor(sorted(fixed.par_st), dtype=torch.long)
        st = _t([fixed.par_st[k] for k in sorted(fixed.par_st)])
        s = s.index_put((idx,), st[:, 0])
        t = t.index_put((idx,), st[:, 1])
    r = r0 + s[:, None] * di - t[:, None] * dj
    dist = torch.sqrt((r * r).sum(1))
    e = r / torch.where(dist > 0, dist, torch.ones_like(dist))[:, None]
    if fixed.degen_e:
        idx = torch.tensor(sorted(fixed.degen_e), dtype=torch.long)
        e = e.index_put((idx,), _t([fixed.degen_e[k] for k in sorted(fixed.degen_e)]))
    return s, t, dist, e


def dense_D_t(n: int, pi, pj, e, dir_, s, t) -> torch.Tensor:
    """D [6n, nc]; column c = [e; y_i x e] on rod i and [-e; -y_j x e] on
    rod j, y = arm * director (eq. blockdef; e points from j to i)."""
    nc = e.shape[0]
    pi_t = torch.as_tensor(pi, dtype=torch.long)
    pj_t = torch.as_tensor(pj, dtype=torch.long)
    yi = s[:, None] * dir_[pi_t]
    yj = t[:, None] * dir_[pj_t]
    ti = torch.linalg.cross(yi, e, dim=1)
    tj = torch.linalg.cross(yj, e, dim=1)
    cols = torch.arange(nc, dtype=torch.long)
    rows, vals, cidx = [], [], []
    for k in range(3):
        rows += [6 * pi_t + k, 6 * pi_t + 3 + k, 6 * pj_t + k, 6 * pj_t + 3 + k]
        vals += [e[:, k], ti[:, k], -e[:, k], -tj[:, k]]
        cidx += [cols] * 4
    D = torch.zeros(6 * n, nc, dtype=_T)
    return D.index_put((torch.cat(rows), torch.cat(cidx)), torch.cat(vals), accumulate=True)


def psi_times_t(quat: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """theta_dot = Psi(theta) Omega = 1/2 [-p.Omega ; s Omega - p x Omega]
    (lab-frame Omega; Section "rigid body kinematics")."""
    s, p = quat[:, 0:1], quat[:, 1:]
    return 0.5 * torch.cat([-(p * w).sum(1, keepdim=True), s * w - torch.linalg.cross(p, w, dim=1)], 1)


@dataclass
class StepParams:
    lengths: np.ndarray
    box: np.ndarray
    diam: float
    eta: float
    dt: float


def solve_U_t(n, dir_, Mt, Mr, D, q, F, active):
    """gamma_A = -Mc_AA^{-1} q_A, gamma = 0 elsewhere; U = M (D gamma + F)."""
    nc = D.shape[1]
    Dr = D.reshape(n, 6, nc)
    MD = torch.cat([torch.einsum("nab,nbc->nac", Mt, Dr[:, :3]),
                    torch.einsum("nab,nbc->nac", Mr, Dr[:, 3:])], 1).reshape(6 * n, nc)
    A = torch.as_tensor(np.nonzero(active)[0], dtype=torch.long)
    gamma = torch.zeros(nc, dtype=_T)
    if A.numel():
        McAA = D[:, A].T @ MD[:, A]
        cond = float(np.linalg.cond(McAA.detach().numpy()))
        if not np.isfinite(cond) or cond > 1e12:
            raise ValueError(f"active block singular (cond {cond:.3g}); the oracle needs a regular A")
        gA = -torch.linalg.solve(McAA, q[A])
        gamma = gamma.index_put((A,), gA)
    G = (D @ gamma).reshape(n, 6) + F
    return apply_M_t(Mt, Mr, G), gamma


def step_t(x, quat, F, fixed: Fixed, p: StepParams):
    """One differentiable step: returns (x + h U_t, normalised theta update,
    U, gamma).  x are the centres the pair list was built on (wrapped)."""
    n = x.shape[0]
    dir_ = directors_t(quat)
    L = _t(p.lengths)
    pi = torch.as_tensor(fixed.pi, dtype=torch.long)
    pj = torch.as_tensor(fixed.pj, dtype=torch.long)
    xj = x[pj] + _t(fixed.shift)
    s, t, dist, e = closest_t(x[pi], dir_[pi], 0.5 * L[pi], xj, dir_[pj], 0.5 * L[pj], fixed)
    phi = dist - p.diam
    Mt, Mr = mobility_t(dir_, p.lengths, p.diam, p.eta)
    D = dense_D_t(n, fixed.pi, fixed.pj, e, dir_, s, t)
    Unc = apply_M_t(Mt, Mr, F)
    q = phi / p.dt + D.T @ Unc.reshape(-1)
    U, gamma = solve_U_t(n, dir_, Mt, Mr, D, q, F, fixed.active)
    x1 = x + p.dt * U[:, :3]
    u = quat + p.dt * psi_times_t(quat, U[:, 3:])
    q1 = u / torch.sqrt((u * u).sum(1, keepdim=True))
    return x1, q1, U, gamma


# --- forward with the oracle's solver, recording what is held fixed ---------

def _fixed_from(x, dir_, lengths, box, pr: Pairs, gamma, g) -> Fixed:
    shift = img_unpack(pr.img).astype(np.float64) * np.asarray(box, dtype=np.float64)
    par_st, degen_e = {}, {}
    for c in np.nonzero(pr.flags & 6)[0]:
        i, j = int(pr.pi[c]), int(pr.pj[c])
        s, t, dist, e, fl = closest(x[i], dir_[i], lengths[i], x[j] + shift[c], dir_[j], lengths[j])
        di, dj = dir_[i], dir_[j]
        if 1.0 - float(np.dot(di, dj)) ** 2 <= EPS_PAR:
            par_st[int(c)] = (s, t)
        if dist < DEGEN_DIST:
            degen_e[int(c)] = e
    return Fixed(pr.pi.astype(np.int64), pr.pj.astype(np.int64), shift, np.asarray(gamma > g), par_st, degen_e)


@dataclass
class Record:
    x: np.ndarray           # wrapped centres at the step start
    quat: np.ndarray
    fixed: Fixed
    U: np.ndarray
    iterations: int
    residual: float


def rollout_forward(x0, quat0, lengths, F_seq, box, diam, cutoff, eta, dt, tol=1e-11,
                    max_iter=200_000) -> (np.ndarray, List[Record]):
    """T steps with the oracle's own pair search and BBPGD.  Returns the
    unwrapped final centres and one record per step."""
    x = np.array(x0, dtype=np.float64)
    xu = x.copy()
    quat = np.array(quat0, dtype=np.float64)
    lengths = np.asarray(lengths, dtype=np.float64)
    box3 = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)).copy()
    recs = []
    for Ft in F_seq:
        Ft = np.ascontiguousarray(Ft, dtype=np.float64)
        d = directors(quat)
        pr = pairs(x, d, lengths, box3, diam, cutoff)
        cs = assemble(x, d, lengths, box3, diam, eta, dt, pr, Ft)
        sr = bbpgd(d, lengths, diam, eta, pr, cs, tol=tol, max_iter=max_iter)
        if sr.status != 0:
            raise RuntimeError(f"oracle BBPGD status {sr.status}")
        U = velocity(d, lengths, diam, eta, pr, cs, sr.gamma, Ft)
        recs.append(Record(x.copy(), quat.copy(), _fixed_from(x, d, lengths, box3, pr, sr.gamma, sr.g), U,
                           sr.iterations, sr.residual))
        integrate(box3, dt, U, x, quat, xu)
    return xu, recs


def rollout_loss(x0, quat0, lengths, F_seq, box, diam, cutoff, eta, dt, tol=1e-11) -> float:
    """Sum of squared unwrapped final centres, by the oracle's forward."""
    xu, _ = rollout_forward(x0, quat0, lengths, F_seq, box, diam, cutoff, eta, dt, tol=tol)
    return float((xu * xu).sum())


@dataclass
class RolloutGrad:
    loss: float
    x0_bar: np.ndarray      # [n, 3]
    quat0_bar: np.ndarray   # [n, 4], tangent to the unit sphere
    F_bar: np.ndarray       # [T, n, 6]
    records: List[Record]


def _tangent(quat: np.ndarray, qbar: np.ndarray) -> np.ndarray:
    qn = quat / np.linalg.norm(quat, axis=1, keepdims=True)
    return qbar - (qbar * qn).sum(1, keepdims=True) * qn


def rollout_grad(x0, quat0, lengths, F_seq, box, diam, cutoff, eta, dt, tol=1e-11) -> RolloutGrad:
    """Gradient of sum |x_unwrapped(T)|^2 with respect to x0, theta0 and the
    per-step forces: the oracle's forward fixes pairs and active sets, the
    dense step above is replayed and differentiated."""
    lengths = np.asarray(lengths, dtype=np.float64)
    box3 = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)).copy()
    xu_T, recs = rollout_forward(x0, quat0, lengths, F_seq, box3, diam, cutoff, eta, dt, tol=tol)
    p = StepParams(lengths, box3, diam, eta, dt)
    x0_t = _t(x0).clone().requires_grad_(True)
    q0_t = _t(quat0).clone().requires_grad_(True)
    F_t = _t(np.asarray(F_seq)).clone().requires_grad_(True)
    xu, quat = x0_t, q0_t
    for k, rec in enumerate(recs):
        # the wrapped centres differ from the unwrapped ones by whole box lengths
        wrap = _t(rec.x - xu.detach().numpy())
        x1, quat, _, _ = step_t(xu + wrap, quat, F_t[k], rec.fixed, p)
        xu = x1 - wrap
    loss = (xu * xu).sum()
    loss.backward()
    return RolloutGrad(float(loss.detach()), x0_t.grad.numpy().copy(),
                       _tangent(np.asarray(quat0, dtype=np.float64), q0_t.grad.numpy()),
                       F_t.grad.numpy().copy(), recs)


def step_grad(x, quat, lengths, F, box, diam, cutoff, eta, dt, x1_bar, quat1_bar, tol=1e-11):
    """Adjoint of one step: given the adjoints of the step's outputs (x', theta'),
    the adjoints of (x, theta, F).  theta_bar is tangent to the unit sphere."""
    lengths = np.asarray(lengths, dtype=np.float64)
    box3 = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)).copy()
    _, recs = rollout_forward(x, quat, lengths, [F], box3, diam, cutoff, eta, dt, tol=tol)
    rec = recs[0]
    p = StepParams(lengths, box3, diam, eta, dt)
    x_t = _t(x).clone().requires_grad_(True)
    q_t = _t(quat).clone().requires_grad_(True)
    F_t = _t(F).clone().requires_grad_(True)
    x1, q1, _, _ = step_t(x_t, q_t, F_t, rec.fixed, p)
    obj = (x1 * _t(x1_bar)).sum() + (q1 * _t(quat1_bar)).sum()
    obj.backward()
    return (x_t.grad.numpy().copy(), _tangent(np.asarray(quat, dtype=np.float64), q_t.grad.numpy()),
            F_t.grad.numpy().copy(), rec)


# --- adjoint of the solve alone ----------------------------------------------

def solve_grad(dir_, lengths, diam, eta, pr: Pairs, cs: Constraints, gamma, g, F, U_bar):
    """Adjoint of U = M (D gamma + F) with gamma the solution for the given
    (dir, e, arm, q, F), q taken as an input of its own.  Returns
    (q_bar [nc], e_bar [nc, 3], arm_bar [nc, 2], F_bar [n, 6], dir_bar [n, 3])."""
    n = dir_.shape[0]
    lengths = np.broadcast_to(np.asarray(lengths, dtype=np.float64), (n,))
    d_t = _t(dir_).clone().requires_grad_(True)
    e_t = _t(cs.e).clone().requires_grad_(True)
    arm_t = _t(cs.arm).clone().requires_grad_(True)
    q_t = _t(cs.q).clone().requires_grad_(True)
    F_t = _t(F).clone().requires_grad_(True)
    Mt, Mr = mobility_t(d_t, lengths, diam, eta)
    D = dense_D_t(n, pr.pi, pr.pj, e_t, d_t, arm_t[:, 0], arm_t[:, 1])
    U, _ = solve_U_t(n, d_t, Mt, Mr, D, q_t, F_t, np.asarray(gamma > g))
    (U * _t(U_bar)).sum().backward()
    return (q_t.grad.numpy().copy(), e_t.grad.numpy().copy(), arm_t.grad.numpy().copy(),
            F_t.grad.numpy().copy(), d_t.grad.numpy().copy())
