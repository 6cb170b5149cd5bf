"""Pins of the oracle's time integration (no GPU): the linearised Euler
update C^{k+1} = C^k + h G U (eq. constrainedeom_euler) against closed forms
for a free rod and against the exact rotation for small steps."""
import math

import numpy as np
import pytest

import oracle
import rodsynth


def test_free_rod_translation_is_exact():
    s = rodsynth.make_system(50, seed=0, box=100.0)
    d = oracle.directors(s.quat)
    U = oracle.apply_mobility(d, 1.0, s.diam, s.eta, s.force)
    x, q = s.x.copy(), s.quat.copy()
    oracle.integrate(s.box, s.dt, U, x, q)
    assert np.allclose(x, s.x + s.dt * U[:, :3], rtol=0, atol=1e-15)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-15)


def test_wrap_into_box_and_unwrapped_copy():
    box = 2.0
    x = np.array([[1.999, 0.0005, 1.0]])
    xu = x.copy()
    q = np.array([[1.0, 0, 0, 0]])
    U = np.array([[20.0, -10.0, 0, 0, 0, 0]])
    oracle.integrate(box, 1e-4, U, x, q, xu)
    assert np.allclose(x, [[0.001, 1.9995, 1.0]], atol=1e-12)
    assert np.allclose(xu, [[2.001, -0.0005, 1.0]], atol=1e-12)
    assert np.all((x >= 0) & (x < box))


def test_rotation_step_closed_form():
    """theta + h Psi(theta) Omega = (1 + h/2 Omega) * theta (quaternion
    product), so after renormalisation one step is exactly a rotation about
    Omega by 2 atan(h |Omega| / 2): the axis is exact and the angle is
    h |Omega| up to O(h^3)."""
    rng = np.random.default_rng(1)
    q0 = rng.standard_normal(4)
    q0 /= np.linalg.norm(q0)
    w = rng.standard_normal(3) * 400.0
    d0 = oracle.directors(q0[None])[0]
    k = w / np.linalg.norm(w)

    def rot(ang):
        return d0 * math.cos(ang) + np.cross(k, d0) * math.sin(ang) + k * np.dot(k, d0) * (1 - math.cos(ang))

    errs = []
    for h in (1e-4, 5e-5, 2.5e-5):
        x = np.zeros((1, 3))
        q = q0[None].copy()
        oracle.integrate(100.0, h, np.r_[0, 0, 0, w][None], x, q)
        d1 = oracle.directors(q)[0]
        assert np.allclose(d1, rot(2 * math.atan(0.5 * h * np.linalg.norm(w))), atol=1e-14)
        errs.append(np.linalg.norm(d1 - rot(np.linalg.norm(w) * h)))
    assert errs[0] / errs[1] == pytest.approx(8.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(8.0, rel=0.05)


def test_overlap_is_reduced_to_order_h():
    """Appendix 'Temporal discretization ...': after a solved step the
    remaining overlap is a linearisation error that shrinks with h."""
    F = np.zeros((2, 6))
    res = []
    for dt in (1e-4, 5e-5):
        s = rodsynth.make_system(2, seed=0, box=50.0, dt=dt)
        s.x[:] = [[10, 10, 10 + 0.02], [10.3, 10, 10]]
        # i along x, j tilted in the x-y plane: an off-centre crossing
        s.quat[0] = np.array([1, 0, 1, 0]) / math.sqrt(2)
        s.quat[1] = np.array([1, -1, 0, 0]) / math.sqrt(2)
        s.force[:] = 0.0
        s.force[0, 2] = -50.0
        r = oracle.step_solve(s)
        assert r.pairs.n == 1 and r.solve.gamma[0] > 0
        x, q = s.x.copy(), s.quat.copy()
        oracle.integrate(s.box, s.dt, r.U, x, q)
        d = oracle.directors(q)
        _, _, dist, _, _ = oracle.closest(x[0], d[0], 1.0, x[1], d[1], 1.0)
        res.append(dist - s.diam)
    assert abs(res[0]) < 1e-3 and abs(res[1]) < abs(res[0])
