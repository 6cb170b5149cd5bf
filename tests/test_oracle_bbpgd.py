"""Pins of the oracle's BBPGD solve and velocities (no GPU): closed-form
one-contact and two-rod solutions, decoupled contacts, exhaustive active-set
enumeration and projected Gauss-Seidel on small systems, and the uniqueness of
U = M(D gamma + F) that the convexity of the QP implies (Appendix "Temporal
discretization and convex quadratic programming": Mc is SPSD)."""
import math

import numpy as np
import pytest

import oracle
import rodsynth
from oracle import crosscheck

DIAM, ETA, DT = 0.025, 0.01, 1e-4


def _quat_for(dvec):
    dvec = np.asarray(dvec, float) / np.linalg.norm(dvec)
    z = np.array([0.0, 0.0, 1.0])
    if np.allclose(dvec, -z):
        return np.array([0.0, 1.0, 0.0, 0.0])
    q = np.r_[1.0 + dvec[2], np.cross(z, dvec)]
    return q / np.linalg.norm(q)


class _Sys:
    def __init__(self, x, dirs, F, box=50.0, L=1.0):
        self.x = np.asarray(x, float)
        self.quat = np.stack([_quat_for(v) for v in dirs])
        self.length = np.full(len(self.x), L)
        self.force = np.asarray(F, float)
        self.box, self.diam, self.cutoff, self.eta, self.dt = box, DIAM, 0.05, ETA, DT

    @property
    def uniform_length(self):
        return float(self.length[0])

    @property
    def n(self):
        return len(self.x)


def _dense_Mc(r):
    s_n = r.dir.shape[0]
    D = oracle.dense_D(r.dir, r.pairs, r.cons)
    Mb = np.zeros((6 * s_n, 6 * s_n))
    for i in range(s_n):
        Mb[6 * i:6 * i + 6, 6 * i:6 * i + 6] = oracle.mobility_block(r.dir[i], 1.0, DIAM, ETA)
    return D, Mb, D.T @ Mb @ D


def test_crossed_rods_pushed_together_closed_form():
    """Two perpendicular rods crossing at their centres, overlapping, pushed
    together along the common normal: one contact with zero lever arms, so
    Mc = a_perp,i + a_perp,j and gamma = max(0, -q/Mc)."""
    gap = -0.005                       # overlap of 5 nm
    h = DIAM + gap
    F = np.zeros((2, 6))
    F[0, 2], F[1, 2] = -2.0, 3.0       # i pushed down, j pushed up (j below i)
    s = _Sys([[5, 5, 5 + h], [5, 5, 5]], [[1, 0, 0], [0, 1, 0]], F)
    r = oracle.step_solve(s)
    assert r.pairs.n == 1
    a = oracle.mobility_coeffs(1.0, DIAM, ETA)
    mc = 2 * a[1]
    q = gap / DT + a[1] * (F[0, 2] - F[1, 2])
    assert r.cons.q[0] == pytest.approx(q, rel=1e-13)
    gamma = max(0.0, -q / mc)
    assert r.solve.gamma[0] == pytest.approx(gamma, rel=1e-12)
    assert r.solve.iterations <= 1
    # after the solve the linearised gap is exactly closed: U_i,z - U_j,z = -gap/h
    assert r.U[0, 2] - r.U[1, 2] == pytest.approx(-gap / DT, rel=1e-12)
    assert r.U[0, 2] == pytest.approx(a[1] * (F[0, 2] + gamma), rel=1e-12)
    assert np.allclose(r.U[:, 3:], 0, atol=1e-12)


def test_separating_rods_have_no_force():
    F = np.zeros((2, 6))
    F[0, 2], F[1, 2] = 2.0, -2.0       # pulled apart
    s = _Sys([[5, 5, 5 + DIAM + 0.01], [5, 5, 5]], [[1, 0, 0], [0, 1, 0]], F)
    r = oracle.step_solve(s)
    assert r.pairs.n == 1 and r.solve.gamma[0] == 0.0 and r.solve.iterations == 0
    assert np.allclose(r.U, oracle.apply_mobility(r.dir, 1.0, DIAM, ETA, F))


def test_t_contact_lever_arm_closed_form():
    """The end of rod j presses on the middle of rod i: the lever arm L/2 of
    rod j adds (L/2)^2 r_perp to Mc when the normal is perpendicular to j."""
    gap = -0.004
    F = np.zeros((2, 6))
    F[1, 0] = -5.0                     # j pushed along -x towards rod i
    # rod i along z; rod j along x with its -x end touching rod i
    xj = [DIAM + gap + 0.5, 0.0, 0.0]
    s = _Sys([[0, 0, 0], xj], [[0, 0, 1], [1, 0, 0]], F)
    s.x += 10.0
    r = oracle.step_solve(s)
    assert r.pairs.n == 1
    a = oracle.mobility_coeffs(1.0, DIAM, ETA)
    # normal along x, parallel to rod j (its end cap) and normal to rod i
    assert np.allclose(np.abs(r.cons.e[0]), [1, 0, 0])
    mc = a[1] + a[0]                   # perpendicular mobility of i, axial of j; no torque
    q = gap / DT - a[0] * 5.0          # j sliding axially towards i closes the gap
    assert r.cons.q[0] == pytest.approx(q, rel=1e-12)
    assert r.solve.gamma[0] == pytest.approx(max(0.0, -q / mc), rel=1e-12)


def test_offset_contact_lever_arm_closed_form():
    """Crossed rods touching off-centre on rod i (arm s on i): the normal is
    perpendicular to both axes, so Mc = 2 a_perp + s^2 r_perp."""
    gap = -0.003
    arm = 0.3
    F = np.zeros((2, 6))
    F[1, 2] = 4.0
    s = _Sys([[10 - arm, 10, 10 + DIAM + gap], [10, 10, 10]], [[1, 0, 0], [0, 1, 0]], F)
    r = oracle.step_solve(s)
    assert r.pairs.n == 1
    a = oracle.mobility_coeffs(1.0, DIAM, ETA)
    assert r.cons.arm[0, 0] == pytest.approx(arm, abs=1e-14)
    assert r.cons.arm[0, 1] == pytest.approx(0.0, abs=1e-14)
    mc = 2 * a[1] + arm * arm * a[2]
    q = gap / DT + a[1] * (0.0 - 4.0)
    assert r.cons.q[0] == pytest.approx(q, rel=1e-12)
    g = max(0.0, -q / mc)
    assert r.solve.gamma[0] == pytest.approx(g, rel=1e-12)
    # the contact torque on i spins it about y: Omega_i = r_perp * (arm x e) gamma
    assert r.U[0, 3:] == pytest.approx(a[2] * np.cross([arm, 0, 0], [0, 0, 1]) * g, rel=1e-12, abs=1e-12)


def test_decoupled_contacts_solve_independently():
    rng = np.random.default_rng(0)
    xs, ds, F = [], [], []
    for k in range(6):
        base = np.array([3.0 * k + 2, 5, 5])
        gap = rng.uniform(-0.01, 0.02)
        xs += [base + [0, 0, DIAM + gap], base]
        ds += [[1, 0, 0], [0, 1, 0]]
    F = rng.standard_normal((12, 6))
    s = _Sys(xs, ds, F)
    r = oracle.step_solve(s)
    assert r.pairs.n == 6
    D, Mb, Mc = _dense_Mc(r)
    assert np.allclose(Mc - np.diag(np.diag(Mc)), 0, atol=1e-12)
    want = np.maximum(0.0, -r.cons.q / np.diag(Mc))
    assert np.allclose(r.solve.gamma, want, rtol=1e-9, atol=1e-9)


def _cluster_system(seed, n=14, box=1.6):
    return rodsynth.make_system(n, seed=seed, box=box)


@pytest.mark.parametrize("seed", range(8))
def test_enumeration_agrees_on_small_systems(seed):
    s = _cluster_system(seed)
    r = oracle.step_solve(s, tol=1e-12)
    if not (1 <= r.pairs.n <= 11):
        pytest.skip(f"{r.pairs.n} constraints")
    assert r.solve.status == oracle.OK
    D, Mb, Mc = _dense_Mc(r)
    sols = crosscheck.enumerate_lcp(Mc, r.cons.q)
    assert sols, "enumeration found no solution"
    scale = np.linalg.norm(r.U)
    for g in sols:
        U = oracle.velocity(r.dir, 1.0, DIAM, ETA, r.pairs, r.cons, g, s.force)
        assert np.linalg.norm(U - r.U) <= 1e-8 * scale


def test_some_small_systems_are_enumerable():
    counts = [oracle.step_solve(_cluster_system(sd)).pairs.n for sd in range(8)]
    assert sum(1 <= c <= 11 for c in counts) >= 4


def test_pgs_agrees_on_medium_system():
    s = rodsynth.make_system(150, seed=3, box=3.0)
    r = oracle.step_solve(s, tol=1e-11)
    assert r.pairs.n > 20 and r.solve.status == oracle.OK
    D, Mb, Mc = _dense_Mc(r)
    g, sweeps, res = crosscheck.pgs(Mc, r.cons.q, tol=1e-11)
    assert res <= 1e-11
    U = oracle.velocity(r.dir, 1.0, DIAM, ETA, r.pairs, r.cons, g, s.force)
    assert np.linalg.norm(U - r.U) <= 1e-7 * np.linalg.norm(r.U)


def test_bbpgd_certificate_and_permutation_invariance():
    s = rodsynth.cfg_small(1)
    r = oracle.step_solve(s)
    assert r.solve.status == oracle.OK and r.solve.residual <= 1e-8
    w = oracle.apply_Mc(r.dir, 1.0, DIAM, ETA, r.pairs, r.cons, r.solve.gamma)
    assert np.abs(np.minimum(r.solve.gamma, w)).max() <= 1e-8
    assert r.solve.gamma.min() >= 0
    # constraint order is irrelevant to U (the solution set is the same)
    perm = np.random.default_rng(0).permutation(r.pairs.n)
    pr2 = oracle.Pairs(r.pairs.pi[perm], r.pairs.pj[perm], r.pairs.img[perm], r.pairs.flags[perm])
    cs2 = oracle.Constraints(r.cons.phi[perm], r.cons.e[perm], r.cons.arm[perm], r.cons.q[perm])
    sr2 = oracle.bbpgd(r.dir, 1.0, DIAM, ETA, pr2, cs2, tol=1e-10)
    U2 = oracle.velocity(r.dir, 1.0, DIAM, ETA, pr2, cs2, sr2.gamma, s.force)
    assert np.linalg.norm(U2 - r.U) <= 1e-6 * np.linalg.norm(r.U)


def test_bbpgd_status_codes():
    s = rodsynth.cfg_small(0)
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, 1.0, s.box, DIAM, 0.05)
    cs = oracle.assemble(s.x, d, 1.0, s.box, DIAM, ETA, DT, pr, s.force)
    sr = oracle.bbpgd(d, 1.0, DIAM, ETA, pr, cs, tol=1e-8, max_iter=1)
    assert sr.status == oracle.NOT_CONVERGED and sr.iterations == 1 and sr.residual > 1e-8
    # warm start from the solution converges at once
    full = oracle.bbpgd(d, 1.0, DIAM, ETA, pr, cs, tol=1e-8)
    again = oracle.bbpgd(d, 1.0, DIAM, ETA, pr, cs, tol=1e-8, gamma0=full.gamma)
    assert again.status == oracle.OK and again.iterations == 0


def test_single_contact_converges_in_one_iteration():
    """With one constraint the projected Cauchy step alpha0 = 1/Mc11 lands on
    the solution."""
    F = np.zeros((2, 6))
    s = _Sys([[5, 5, 5 + DIAM - 0.01], [5.2, 5, 5]], [[1, 0, 0], [0, 1, 0]], F)
    r = oracle.step_solve(s)
    assert r.pairs.n == 1 and r.solve.iterations == 1
    D, Mb, Mc = _dense_Mc(r)
    assert r.solve.alpha0 == pytest.approx(1.0 / Mc[0, 0], rel=1e-14)
    assert r.solve.gamma[0] == pytest.approx(-r.cons.q[0] / Mc[0, 0], rel=1e-13)


def test_timing_build_agrees_with_the_checker():
    """The CPU baseline times the same oracle source built -O3 -march=native
    (contractions allowed); its solution must agree with the checker build's
    to rounding: both certified, the same unique U."""
    s = rodsynth.cfg_small(2)
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, s.force)
    ref = oracle.bbpgd(d, 1.0, s.diam, s.eta, pr, cs, tol=1e-10)
    Uref = oracle.velocity(d, 1.0, s.diam, s.eta, pr, cs, ref.gamma, s.force)
    prev = oracle.use_build("timing")
    try:
        r = oracle.bbpgd(d, 1.0, s.diam, s.eta, pr, cs, tol=1e-10)
        U = oracle.velocity(d, 1.0, s.diam, s.eta, pr, cs, r.gamma, s.force)
    finally:
        oracle.use_build(prev)
    assert ref.status == oracle.OK and r.status == oracle.OK
    assert np.linalg.norm(U - Uref) <= 1e-9 * np.linalg.norm(Uref)
