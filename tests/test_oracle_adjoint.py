"""Pins of the oracle gradient (CPU).

The oracle differentiates a dense re-statement of the step (fixed pairs and
active set) with PyTorch autograd.  These tests tie it to things outside
itself:
  * central differences of the C oracle's own forward (pair search, BBPGD to
    1e-11, Euler update) on the 20-rod periodic system at volume fraction
    0.05, over a two-step rollout;
  * closed forms for two crossed rods in contact (one active constraint);
  * central differences of the C oracle's BBPGD for the adjoint of the
    solve alone (q, e, arm, F and the directors as inputs).
"""
import numpy as np
import pytest

import oracle
import rodsynth
from oracle import adjoint as adj


def _fd20():
    s = rodsynth.make_system(20, seed=0, phi=0.05)
    rng = np.random.default_rng(11)
    F = np.stack([s.force, rng.standard_normal(s.force.shape)])
    return s, F


def _loss(s, F, x0=None, q0=None):
    return adj.rollout_loss(s.x if x0 is None else x0, s.quat if q0 is None else q0, s.length, F, s.box,
                            s.diam, s.cutoff, s.eta, s.dt)


def _actives(s, F, x0=None, q0=None):
    _, recs = adj.rollout_forward(s.x if x0 is None else x0, s.quat if q0 is None else q0, s.length, F, s.box,
                                  s.diam, s.cutoff, s.eta, s.dt)
    return [(r.fixed.pi.tobytes(), r.fixed.pj.tobytes(), r.fixed.active.tobytes()) for r in recs]


def _rotate(quat, omega):
    """theta rotated by the small lab-frame rotation vector omega, normalised."""
    s, p = quat[:, :1], quat[:, 1:]
    dq = 0.5 * np.concatenate([-(omega * p).sum(1, keepdims=True), s * omega + np.cross(omega, p)], 1)
    q = quat + dq
    return q / np.linalg.norm(q, axis=1, keepdims=True)


@pytest.fixture(scope="module")
def fd_case():
    s, F = _fd20()
    g = adj.rollout_grad(s.x, s.quat, s.length, F, s.box, s.diam, s.cutoff, s.eta, s.dt)
    return s, F, g


def test_replay_matches_oracle_forward(fd_case):
    """The dense differentiable replay reproduces the oracle's trajectory."""
    import torch
    s, F, g = fd_case
    p = adj.StepParams(s.length, np.full(3, s.box), s.diam, s.eta, s.dt)
    xu = s.x.copy()
    quat = torch.as_tensor(s.quat)
    for k, rec in enumerate(g.records):
        wrap = rec.x - xu
        x1, quat, U, _ = adj.step_t(torch.as_tensor(rec.x), quat, torch.as_tensor(F[k]), rec.fixed, p)
        assert np.allclose(U.numpy(), rec.U, rtol=0, atol=1e-7 * np.abs(rec.U).max())
        xu = x1.numpy() - wrap
    xu_oracle, _ = adj.rollout_forward(s.x, s.quat, s.length, F, s.box, s.diam, s.cutoff, s.eta, s.dt)
    assert np.allclose(xu, xu_oracle, rtol=0, atol=1e-12)
    assert g.records[0].fixed.active.sum() > 20


@pytest.mark.parametrize("what", ["F", "x0", "theta0"])
def test_gradient_matches_central_differences(fd_case, what):
    s, F, g = fd_case
    rng = np.random.default_rng({"F": 1, "x0": 2, "theta0": 3}[what])
    base = _actives(s, F)
    eps = 1e-6
    for _ in range(4):
        if what == "F":
            v = rng.standard_normal(F.shape)
            lp, lm = _loss(s, F + eps * v), _loss(s, F - eps * v)
            assert _actives(s, F + eps * v) == base and _actives(s, F - eps * v) == base
            an = float((g.F_bar * v).sum())
        elif what == "x0":
            v = rng.standard_normal(s.x.shape)
            lp, lm = _loss(s, F, x0=s.x + eps * v), _loss(s, F, x0=s.x - eps * v)
            assert _actives(s, F, x0=s.x + eps * v) == base
            an = float((g.x0_bar * v).sum())
        else:
            w = rng.standard_normal(s.x.shape)
            qp, qm = _rotate(s.quat, eps * w), _rotate(s.quat, -eps * w)
            lp, lm = _loss(s, F, q0=qp), _loss(s, F, q0=qm)
            assert _actives(s, F, q0=qp) == base
            # the directional derivative along the rotation: theta_bar . (1/2 (0, w) theta)
            sq, pq = s.quat[:, :1], s.quat[:, 1:]
            dq = 0.5 * np.concatenate([-(w * pq).sum(1, keepdims=True), sq * w + np.cross(w, pq)], 1)
            an = float((g.quat0_bar * dq).sum())
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9, (what, fd, an)


def _crossed(overlap=0.004):
    """Rod i along x above rod j along y, axes crossing at their centres,
    axis distance diam - overlap: one active contact with normal +z."""
    diam = rodsynth.DIAM
    x = np.array([[5.0, 5.0, 5.0 + diam - overlap], [5.0, 5.0, 5.0]])
    quat = np.array([[np.cos(np.pi / 4), 0.0, np.sin(np.pi / 4), 0.0],     # z -> x
                     [np.cos(np.pi / 4), -np.sin(np.pi / 4), 0.0, 0.0]])   # z -> y
    return x, quat


def test_closed_form_crossed_rods_step():
    """One active contact between crossed rods touching at their centres:
    the Euler step closes the gap exactly, each rod moving half of it, so
    d(x1_i.e)/d(x_i.e) = d(x1_i.e)/d(x_j.e) = 1/2; and along e each rod takes
    half of either external force: d(x1_i.e)/d(F.e) = h a_perp / 2."""
    x, quat = _crossed()
    d = oracle.directors(quat)
    assert np.allclose(d, [[1, 0, 0], [0, 1, 0]], atol=1e-15)
    L, diam, eta, dt = np.ones(2), rodsynth.DIAM, rodsynth.ETA, rodsynth.DT
    F = np.zeros((2, 6))
    x1_bar = np.zeros((2, 3))
    x1_bar[0, 2] = 1.0
    xb, qb, Fb, rec = adj.step_grad(x, quat, L, F, 10.0, diam, 0.05, eta, dt, x1_bar, np.zeros((2, 4)))
    assert rec.fixed.active.tolist() == [True]
    aperp = oracle.mobility_coeffs(1.0, diam, eta)[1]
    assert xb[0, 2] == pytest.approx(0.5, rel=1e-12)
    assert xb[1, 2] == pytest.approx(0.5, rel=1e-12)
    assert Fb[0, 2] == pytest.approx(dt * aperp / 2, rel=1e-12)
    assert Fb[1, 2] == pytest.approx(dt * aperp / 2, rel=1e-12)
    # tangential motion of the contact does not change the normal response
    assert np.allclose(xb[:, :2], 0.0, atol=1e-12)


def test_closed_form_single_contact_solve():
    """Adjoint of the solve alone at one active contact: gamma = -q / Mc_11,
    so q_bar = -(d^T M U_bar) / Mc_11; with U_bar the unit normal velocity of
    rod i that is -a_perp / (2 a_perp) = -1/2, and F_bar = M U_bar."""
    x, quat = _crossed()
    d = oracle.directors(quat)
    L, diam, eta, dt = 1.0, rodsynth.DIAM, rodsynth.ETA, rodsynth.DT
    F = np.zeros((2, 6))
    pr = oracle.pairs(x, d, L, 10.0, diam, 0.05)
    cs = oracle.assemble(x, d, L, 10.0, diam, eta, dt, pr, F)
    sr = oracle.bbpgd(d, L, diam, eta, pr, cs, tol=1e-13)
    Ub = np.zeros((2, 6))
    Ub[0, 2] = 1.0
    qb, eb, ab, Fb, db = adj.solve_grad(d, L, diam, eta, pr, cs, sr.gamma, sr.g, F, Ub)
    aperp = oracle.mobility_coeffs(1.0, diam, eta)[1]
    assert qb[0] == pytest.approx(-0.5, rel=1e-12)
    assert np.allclose(Fb, aperp * Ub, rtol=1e-13, atol=1e-12 * aperp)


def test_solve_adjoint_matches_central_differences():
    """Directional derivatives of U_bar . U with the oracle's BBPGD (to
    1e-13) re-run at perturbed inputs."""
    s = rodsynth.make_system(20, seed=0, phi=0.05)
    d = oracle.directors(s.quat)
    L = s.uniform_length
    pr = oracle.pairs(s.x, d, L, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, L, s.box, s.diam, s.eta, s.dt, pr, s.force)
    sr = oracle.bbpgd(d, L, s.diam, s.eta, pr, cs, tol=1e-12)
    rng = np.random.default_rng(4)
    Ub = rng.standard_normal((s.n, 6))
    qb, eb, ab, Fb, db = adj.solve_grad(d, L, s.diam, s.eta, pr, cs, sr.gamma, sr.g, s.force, Ub)
    act = sr.gamma > sr.g

    def J(dd=d, e=cs.e, arm=cs.arm, q=cs.q, F=s.force):
        c2 = oracle.Constraints(cs.phi, np.ascontiguousarray(e), np.ascontiguousarray(arm), np.ascontiguousarray(q))
        r = oracle.bbpgd(dd, L, s.diam, s.eta, pr, c2, tol=1e-13)
        assert ((r.gamma > r.g) == act).all()
        return float((Ub * oracle.velocity(dd, L, s.diam, s.eta, pr, c2, r.gamma, F)).sum())

    eps = 1e-6
    for name, base, grad in [("q", cs.q, qb), ("e", cs.e, eb), ("arm", cs.arm, ab), ("F", s.force, Fb),
                             ("dir", d, db)]:
        v = rng.standard_normal(base.shape)
        fd = (J(**{{"q": "q", "e": "e", "arm": "arm", "F": "F", "dir": "dd"}[name]: base + eps * v})
              - J(**{{"q": "q", "e": "e", "arm": "arm", "F": "F", "dir": "dd"}[name]: base - eps * v})) / (2 * eps)
        an = float((grad * v).sum())
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-8, (name, fd, an)
