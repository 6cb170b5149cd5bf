"""When the linearised step has a solution (CPU, oracle only).

The problem of eq. cqpdef is min f(g) = 1/2 g.Mc g + q.g over g >= 0 with
Mc = D^T M D (block B of eq. blockdef) and q = phi/h + D^T M F (block A).
Mc is only semi-definite, so f may be unbounded below.  Along a direction
d >= 0, f(t d) = t^2/2 d.Mc d + t q.d; d.Mc d = |M^(1/2) D d|^2 vanishes
exactly when D d = 0 (M is positive definite), and then q.d = phi.d / h.
Hence:
  * if every gap phi >= 0, no such direction lowers f, the convex QP is
    bounded below and attains its minimum: the complementarity problem is
    solvable;
  * if some d >= 0 has D d = 0 and phi.d < 0, then for every g >= 0,
    d.(Mc g + q) = (D d).M D g + phi.d / h = phi.d / h < 0, so w = Mc g + q
    cannot be >= 0 everywhere: no solution exists (a Farkas certificate).
Random isotropic rods at volume fraction 0.08 with lengths in [0.5, 1.5]
overlap enough for such a d to exist; these tests find one with a linear
program, check it against the oracle's own operator, and show the oracle's
BBPGD iterates running down that ray.  The same geometry with every gap made
non-negative solves.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import oracle
import rodsynth


def _unrelaxed(n=300, seed=0):
    s = rodsynth.make_system(n, seed=seed, phi=0.08, length=(0.5, 1.5), orientation="isotropic")
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, s.length, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, s.length, s.box, s.diam, s.eta, s.dt, pr, s.force)
    return s, d, pr, cs


@pytest.fixture(scope="module")
def dense():
    return _unrelaxed()


def test_unrelaxed_dense_problem_has_an_infeasibility_certificate(dense):
    s, d, pr, cs = dense
    assert (cs.phi < 0).sum() > 0.25 * pr.n  # about one overlap per rod pair in four
    D = sp.csc_matrix(oracle.dense_D(d, pr, cs))
    # find z >= 0 with D z = 0 and phi.z = -1 (minimising sum z for a sparse one)
    A = sp.vstack([D, sp.csr_matrix(cs.phi.reshape(1, -1))]).tocsc()
    b = np.zeros(D.shape[0] + 1)
    b[-1] = -1.0
    res = linprog(np.ones(pr.n), A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    z = np.maximum(res.x, 0.0)
    assert abs(cs.phi @ z + 1.0) < 1e-9
    # the oracle's operator: Mc z = D^T M D z vanishes, q.z = phi.z / h
    Mz = oracle.apply_Mc(d, s.length, s.diam, s.eta, pr, cs, z, add_q=False)
    assert np.abs(Mz).max() < 1e-6 * np.abs(cs.q).max()
    assert abs(cs.q @ z * s.dt + 1.0) < 1e-6
    # so z.w = z.(Mc g + q) < 0 for the oracle's iterates: w >= 0 is impossible
    r = oracle.bbpgd(d, s.length, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=2000)
    w = oracle.apply_Mc(d, s.length, s.diam, s.eta, pr, cs, r.gamma)
    assert z @ w < -0.99 / s.dt
    assert r.status == oracle.NOT_CONVERGED and np.min(w) < -1e-8


def test_bbpgd_runs_down_the_unbounded_ray(dense):
    s, d, pr, cs = dense
    prev_f, prev_c = 0.0, np.inf
    for it in (500, 2000, 8000):
        r = oracle.bbpgd(d, s.length, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=it)
        assert r.status == oracle.NOT_CONVERGED
        w = oracle.apply_Mc(d, s.length, s.diam, s.eta, pr, cs, r.gamma)
        f = 0.5 * r.gamma @ (w + cs.q)
        u = r.gamma / np.linalg.norm(r.gamma)
        curv = u @ oracle.apply_Mc(d, s.length, s.diam, s.eta, pr, cs, u, add_q=False)
        # the objective keeps falling, the direction's curvature goes to 0
        # while its gap product stays negative
        assert f < 2.5 * prev_f - 1e6
        assert curv < 0.5 * prev_c
        assert cs.phi @ u < -0.05
        prev_f, prev_c = f, curv


def test_nonnegative_gaps_always_solve(dense):
    s, d, pr, cs = dense
    # same D (same Mc), every gap replaced by its magnitude: q' = |phi|/h + D^T M F
    q2 = cs.q + (np.abs(cs.phi) - cs.phi) / s.dt
    cs2 = oracle.Constraints(cs.phi, cs.e, cs.arm, q2)
    r = oracle.bbpgd(d, s.length, s.diam, s.eta, pr, cs2, tol=1e-8, max_iter=100_000)
    assert r.status == oracle.OK and r.residual <= 1e-8
    w = oracle.apply_Mc(d, s.length, s.diam, s.eta, pr, cs2, r.gamma)
    assert r.gamma.min() >= 0.0 and w.min() >= -1e-8 and np.abs(r.gamma * w).max() <= 1e-6
