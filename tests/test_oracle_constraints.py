"""Pins of the oracle's constraint geometry, its constraint-space operator and
its velocity (no GPU).

The main pin is the identity grad_C Phi . G = D^T of eq. (symmetrydmap): the
rate of change of every gap under a rigid motion of the rods equals the
D-matrix column dotted with the rods' velocities.  It is checked by central
differences of the gap itself (recomputed from scratch by the closest-point
routine), so a wrong sign, lever arm, cross product or normal fails it."""
import numpy as np
import pytest

import oracle
import rodsynth


@pytest.fixture(scope="module")
def small():
    s = rodsynth.cfg_small(0)
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, s.force)
    return s, d, pr, cs


def _moved(s, V, eps):
    """Configuration after time eps at rod velocities V = [U, Omega] (first order
    in eps for the quaternion, renormalised)."""
    x = s.x + eps * V[:, :3]
    q = s.quat.copy()
    for i in range(s.n):
        q[i] = q[i] + eps * oracle.psi_times(q[i], V[i, 3:])
        q[i] /= np.linalg.norm(q[i])
    return x, q


def _gaps(x, quat, s, pr, idx):
    d = oracle.directors(quat)
    imgs = oracle.img_unpack(pr.img)
    out = []
    for k in idx:
        i, j = pr.pi[k], pr.pj[k]
        _, _, dist, _, _ = oracle.closest(x[i], d[i], 1.0, x[j] + imgs[k] * s.box, d[j], 1.0)
        out.append(dist - s.diam)
    return np.array(out)


def test_D_columns_are_gap_gradients(small):
    s, d, pr, cs = small
    rng = np.random.default_rng(0)
    V = rng.standard_normal((s.n, 6))
    D = oracle.dense_D(d, pr, cs)
    # skip pairs whose closest point sits at a kink of the gap function
    idx = [k for k in range(pr.n) if not pr.flags[k]][:300]
    eps = 1e-7
    xp, qp = _moved(s, V, eps)
    xm, qm = _moved(s, V, -eps)
    fd = (_gaps(xp, qp, s, pr, idx) - _gaps(xm, qm, s, pr, idx)) / (2 * eps)
    an = D[:, idx].T @ V.reshape(-1)
    assert np.allclose(fd, an, rtol=1e-5, atol=1e-6 * np.abs(V).max())


def test_force_and_torque_balance_per_column(small):
    s, d, pr, cs = small
    D = oracle.dense_D(d, pr, cs)
    imgs = oracle.img_unpack(pr.img)
    for k in range(0, pr.n, 7):
        i, j = pr.pi[k], pr.pj[k]
        col = D[:, k].reshape(s.n, 6)
        if i == j:
            continue
        Fi, Ti, Fj, Tj = col[i, :3], col[i, 3:], col[j, :3], col[j, 3:]
        assert np.allclose(Fi + Fj, 0, atol=1e-15)
        # total torque about the origin vanishes: forces act along the line of centres of action
        xj = s.x[j] + imgs[k] * s.box
        tot = np.cross(s.x[i], Fi) + Ti + np.cross(xj, Fj) + Tj
        assert np.allclose(tot, 0, atol=1e-12)
        # the normal is a unit vector pointing from j to i, gap = distance - diam
        assert np.linalg.norm(Fi) == pytest.approx(1.0, abs=1e-14)


def test_q_is_gap_rate_under_free_motion(small):
    """q = phi/h + D^T M F (eq. blockdef, block A): h*q - phi is h times the
    rate of change of the gap when the rods move at U_nc = M F."""
    s, d, pr, cs = small
    Unc = oracle.apply_mobility(d, 1.0, s.diam, s.eta, s.force)
    idx = [k for k in range(pr.n) if not pr.flags[k]][:200]
    eps = 1e-8
    xp, qp = _moved(s, Unc, eps)
    xm, qm = _moved(s, Unc, -eps)
    rate = (_gaps(xp, qp, s, pr, idx) - _gaps(xm, qm, s, pr, idx)) / (2 * eps)
    want = cs.phi[idx] / s.dt + rate
    assert np.allclose(cs.q[idx], want, rtol=1e-5, atol=1e-4)


def test_zero_force_q_is_phi_over_h(small):
    s, d, pr, cs = small
    cs0 = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, np.zeros_like(s.force))
    assert np.array_equal(cs0.q, cs0.phi / s.dt)
    assert np.array_equal(cs0.phi, cs.phi)


def test_Mc_symmetric_psd_and_dense_agrees(small):
    s, d, pr, cs = small
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal(pr.n), rng.standard_normal(pr.n)
    Mu = oracle.apply_Mc(d, 1.0, s.diam, s.eta, pr, cs, u, add_q=False)
    Mv = oracle.apply_Mc(d, 1.0, s.diam, s.eta, pr, cs, v, add_q=False)
    assert np.dot(u, Mv) == pytest.approx(np.dot(v, Mu), rel=1e-13)
    assert np.dot(u, Mu) > 0
    # against D^T M D formed densely with the 6x6 blocks
    D = oracle.dense_D(d, pr, cs)
    Mb = np.zeros((6 * s.n, 6 * s.n))
    for i in range(s.n):
        Mb[6 * i:6 * i + 6, 6 * i:6 * i + 6] = oracle.mobility_block(d[i], 1.0, s.diam, s.eta)
    Mc = D.T @ Mb @ D
    assert np.allclose(Mc @ u, Mu, rtol=1e-12, atol=1e-10 * np.abs(Mu).max())
    w = oracle.apply_Mc(d, 1.0, s.diam, s.eta, pr, cs, u, add_q=True)
    assert np.allclose(w, Mu + cs.q, rtol=1e-14, atol=1e-12)


def test_Mc_diagonal_closed_form(small):
    s, d, pr, cs = small
    c = oracle.mobility_coeffs(1.0, s.diam, s.eta)
    for k in range(0, pr.n, 11):
        i, j = pr.pi[k], pr.pj[k]
        if i == j:
            continue
        e = cs.e[k]
        unit = np.zeros(pr.n)
        unit[k] = 1.0
        mkk = oracle.apply_Mc(d, 1.0, s.diam, s.eta, pr, cs, unit, add_q=False)[k]
        want = 0.0
        for rod, arm in ((i, cs.arm[k, 0]), (j, cs.arm[k, 1])):
            ed = np.dot(e, d[rod])
            want += c[1] + (c[0] - c[1]) * ed * ed            # e . M_t e
            t = arm * np.cross(d[rod], e)                     # lever arm torque, normal to the axis
            want += c[2] * np.dot(t, t)
        assert mkk == pytest.approx(want, rel=1e-13)


def test_velocity_is_mobility_times_total_force(small):
    s, d, pr, cs = small
    rng = np.random.default_rng(2)
    gamma = np.abs(rng.standard_normal(pr.n))
    U = oracle.velocity(d, 1.0, s.diam, s.eta, pr, cs, gamma, s.force)
    D = oracle.dense_D(d, pr, cs)
    Ft = (D @ gamma).reshape(s.n, 6) + s.force
    assert np.allclose(U, oracle.apply_mobility(d, 1.0, s.diam, s.eta, Ft), rtol=1e-13, atol=1e-11)
    # no contacts: U = M F
    empty = oracle.Pairs(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint8))
    ce = oracle.Constraints(np.zeros(0), np.zeros((0, 3)), np.zeros((0, 2)), np.zeros(0))
    U0 = oracle.velocity(d, 1.0, s.diam, s.eta, empty, ce, np.zeros(0), s.force)
    assert np.array_equal(U0, oracle.apply_mobility(d, 1.0, s.diam, s.eta, s.force))
