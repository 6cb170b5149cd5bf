"""Dense cross-check solvers for tiny systems (test infrastructure only).

Both solve the linear complementarity problem that the constraint step
reduces to: gamma >= 0, w = Mc gamma + q >= 0, gamma . w = 0, which is the
KKT system of the convex QP of eq. (suppcqpdef) (Appendix "Temporal
discretization and convex quadratic programming").  They are different
algorithms from the oracle's BBPGD and so check it independently:

* ``enumerate_lcp``: every active set A; gamma_A from Mc_AA gamma_A = -q_A
  (least squares, so singular Mc_AA is allowed), gamma = 0 elsewhere; keep the
  sets that satisfy all complementarity conditions.
* ``pgs``: projected Gauss-Seidel on the explicitly formed Mc.
"""
from __future__ import annotations

import itertools

import numpy as np


def enumerate_lcp(Mc: np.ndarray, q: np.ndarray, tol: float = 1e-10):
    """All solutions found by active-set enumeration (len(q) <= ~12)."""
    nc = q.shape[0]
    scale = max(1.0, float(np.abs(q).max(initial=0.0)))
    sols = []
    for k in range(nc + 1):
        for A in itertools.combinations(range(nc), k):
            A = list(A)
            gamma = np.zeros(nc)
            if A:
                sub = Mc[np.ix_(A, A)]
                gA, *_ = np.linalg.lstsq(sub, -q[A], rcond=None)
                gamma[A] = gA
            w = Mc @ gamma + q
            if gamma.min(initial=0.0) < -tol * scale:
                continue
            if A and np.abs(w[A]).max() > tol * scale:
                continue
            inactive = [c for c in range(nc) if c not in A]
            if inactive and w[inactive].min() < -tol * scale:
                continue
            sols.append(np.maximum(gamma, 0.0))
    return sols


def pgs(Mc: np.ndarray, q: np.ndarray, tol: float = 1e-10, max_sweeps: int = 200_000):
    """Projected Gauss-Seidel; returns (gamma, sweeps, residual)."""
    nc = q.shape[0]
    gamma = np.zeros(nc)
    w = q.copy()
    diag = np.diag(Mc).copy()
    res = np.inf
    for sweep in range(1, max_sweeps + 1):
        for c in range(nc):
            if diag[c] <= 0.0:
                continue
            new = max(0.0, gamma[c] - w[c] / diag[c])
            delta = new - gamma[c]
            if delta != 0.0:
                w += Mc[:, c] * delta
                gamma[c] = new
        w = Mc @ gamma + q
        res = float(np.abs(np.minimum(gamma, w)).max(initial=0.0))
        if res <= tol:
            return gamma, sweep, res
    return gamma, max_sweeps, res
