"""Parity of the differentiation form (rl_solve_lcp_adjoint, rl_step_adjoint,
the checkpointed rollout) with the oracle gradient.

The oracle differentiates the dense active-set statement of the step on the
CPU (pinned by central differences of the oracle's own BBPGD).  Bar: each
gradient array within 1e-6 of its largest magnitude.  That is the relative
bar of the velocities U, and every gradient here is a linear functional
of U-like quantities solved to the same tolerances (forward residual 1e-10,
CG 1e-12 relative).  The active set must match exactly: the zero pattern of
q_bar = -lambda.
"""
import numpy as np
import pytest

import oracle
import rodsynth
from oracle import adjoint as adj

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"
BAR = 1e-6
SYSTEMS = {
    "fd20": lambda: rodsynth.make_system(20, seed=0, phi=0.05),
    "rods200": lambda: rodsynth.make_system(200, seed=2, phi=0.04),
    "lengths": lambda: rodsynth.make_system(300, seed=1, phi=0.04, length=(0.5, 1.5)),
}


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _solver(rl, s, **kw):
    kw.setdefault("tol", 1e-10)
    kw.setdefault("max_iter", 400_000)
    return rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, **kw)


def _glen(s):
    return s.uniform_length if s.uniform_length is not None else _t(s.length)


def _close(name, got, want, bar=BAR):
    got, want = np.asarray(got), np.asarray(want)
    scale = max(np.abs(want).max(), 1e-300)
    err = np.abs(got - want).max() / scale
    print(f"  {name}: max |err| / max |ref| = {err:.3e}", flush=True)
    assert err <= bar, (name, err)


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_solve_adjoint_matches_oracle(gpu_lib, name):
    s = SYSTEMS[name]()
    L = s.uniform_length if s.uniform_length is not None else s.length
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, L, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, L, s.box, s.diam, s.eta, s.dt, pr, s.force)
    sr = oracle.bbpgd(d, L, s.diam, s.eta, pr, cs, tol=1e-11, max_iter=400_000)
    assert sr.status == oracle.OK
    Ub = np.random.default_rng(7).standard_normal((s.n, 6))
    want = adj.solve_grad(d, L, s.diam, s.eta, pr, cs, sr.gamma, sr.g, s.force, Ub)
    with _solver(gpu_lib, s) as slv:
        args = (_t(d), _glen(s), _t(pr.pi, torch.int32), _t(pr.pj, torch.int32), _t(cs.e), _t(cs.arm), _t(cs.q))
        gamma, U, info = slv.solve_lcp(*args, F=_t(s.force))
        assert info.status == 0
        qb, eb, ab, Fb, db, ai = slv.solve_lcp_adjoint(*args, gamma, _t(Ub), F=_t(s.force), cg_tol=1e-12)
    print(f"{name}: nc {pr.n}, active {ai.n_active}, CG {ai.cg_iterations} it, rel res {ai.cg_residual:.2e}")
    assert ai.status == 0
    qb = qb.cpu().numpy()
    assert ai.n_active == int((sr.gamma > sr.g).sum())
    assert np.array_equal(qb != 0.0, want[0] != 0.0)
    for nm, g, w in zip(("q_bar", "e_bar", "arm_bar", "F_bar", "dir_bar"),
                        (qb, eb.cpu().numpy(), ab.cpu().numpy(), Fb.cpu().numpy(), db.cpu().numpy()), want):
        _close(nm, g, w)


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_step_adjoint_matches_oracle(gpu_lib, name):
    s = SYSTEMS[name]()
    rng = np.random.default_rng(8)
    xb1 = rng.standard_normal((s.n, 3))
    qb1 = rng.standard_normal((s.n, 4))
    xb, qb, Fb, rec = adj.step_grad(s.x, s.quat, s.length, s.force, s.box, s.diam, s.cutoff, s.eta, s.dt, xb1, qb1)
    with _solver(gpu_lib, s) as slv:
        x_bar, q_bar = _t(xb1), _t(qb1)
        F_bar, ai = slv.step_adjoint(_t(s.x), _t(s.quat), _glen(s), _t(s.force), x_bar, q_bar, cg_tol=1e-12)
    print(f"{name}: active {ai.n_active} (oracle {int(rec.fixed.active.sum())}), CG {ai.cg_iterations} it, "
          f"forward {ai.solve_iterations} it")
    assert ai.status == 0 and ai.solve_status == 0
    assert ai.n_active == int(rec.fixed.active.sum())
    _close("x_bar", x_bar.cpu().numpy(), xb)
    _close("quat_bar", q_bar.cpu().numpy(), qb)
    _close("F_bar", F_bar.cpu().numpy(), Fb)


def test_crossed_rods_closed_form(gpu_lib):
    """One active contact between crossed rods touching at their centres:
    d(x1_i.e)/d(x_i.e) = d(x1_i.e)/d(x_j.e) = 1/2 and d(x1_i.e)/d(F.e) =
    h a_perp / 2 for either rod."""
    diam = rodsynth.DIAM
    x = np.array([[5.0, 5.0, 5.0 + diam - 0.004], [5.0, 5.0, 5.0]])
    quat = np.array([[np.cos(np.pi / 4), 0.0, np.sin(np.pi / 4), 0.0],
                     [np.cos(np.pi / 4), -np.sin(np.pi / 4), 0.0, 0.0]])
    s = rodsynth.RodSystem(x=x, quat=quat, length=np.ones(2), force=np.zeros((2, 6)), box=10.0)
    xb1 = np.zeros((2, 3))
    xb1[0, 2] = 1.0
    with _solver(gpu_lib, s) as slv:
        x_bar, q_bar = _t(xb1), _t(np.zeros((2, 4)))
        F_bar, ai = slv.step_adjoint(_t(x), _t(quat), 1.0, _t(s.force), x_bar, q_bar)
    aperp = oracle.mobility_coeffs(1.0, diam, rodsynth.ETA)[1]
    xb, Fb = x_bar.cpu().numpy(), F_bar.cpu().numpy()
    assert ai.n_active == 1
    assert xb[0, 2] == pytest.approx(0.5, rel=1e-12) and xb[1, 2] == pytest.approx(0.5, rel=1e-12)
    assert Fb[0, 2] == pytest.approx(rodsynth.DT * aperp / 2, rel=1e-12)
    assert Fb[1, 2] == pytest.approx(rodsynth.DT * aperp / 2, rel=1e-12)


def test_free_rods(gpu_lib):
    """No contacts: lambda is empty, x_bar passes through and F_bar = h M x_bar'."""
    s = rodsynth.make_system(50, seed=3, box=40.0)
    rng = np.random.default_rng(9)
    xb1 = rng.standard_normal((s.n, 3))
    xb, qb, Fb, rec = adj.step_grad(s.x, s.quat, s.length, s.force, s.box, s.diam, s.cutoff, s.eta, s.dt, xb1,
                                    np.zeros((s.n, 4)))
    assert rec.fixed.pi.size == 0
    with _solver(gpu_lib, s) as slv:
        x_bar, q_bar = _t(xb1), _t(np.zeros((s.n, 4)))
        F_bar, ai = slv.step_adjoint(_t(s.x), _t(s.quat), 1.0, _t(s.force), x_bar, q_bar)
    assert ai.n_active == 0 and ai.cg_iterations == 0
    assert np.array_equal(x_bar.cpu().numpy(), xb1)
    _close("F_bar", F_bar.cpu().numpy(), Fb, 1e-13)
    _close("quat_bar", q_bar.cpu().numpy(), qb, 1e-12)


def test_empty(gpu_lib):
    s = rodsynth.make_system(4, seed=0, box=10.0)
    with _solver(gpu_lib, s) as slv:
        e = torch.empty((0, 3), dtype=torch.float64, device=DEV)
        F_bar, ai = slv.step_adjoint(e, torch.empty((0, 4), dtype=torch.float64, device=DEV), 1.0,
                                     torch.empty((0, 6), dtype=torch.float64, device=DEV), e.clone(),
                                     torch.empty((0, 4), dtype=torch.float64, device=DEV))
    assert ai.status == 0 and F_bar.shape == (0, 6)


def test_step_adjoint_is_bitwise_repeatable(gpu_lib):
    s = SYSTEMS["rods200"]()
    rng = np.random.default_rng(10)
    xb1, qb1 = rng.standard_normal((s.n, 3)), rng.standard_normal((s.n, 4))
    outs = []
    with _solver(gpu_lib, s) as slv:
        for _ in range(2):
            x_bar, q_bar = _t(xb1), _t(qb1)
            F_bar, _ = slv.step_adjoint(_t(s.x), _t(s.quat), 1.0, _t(s.force), x_bar, q_bar)
            outs.append([v.cpu().numpy() for v in (x_bar, q_bar, F_bar)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def _gpu_rollout_grad(rl, s, F, k):
    from paper_2109_08206_amd.rollout import rollout
    with _solver(rl, s) as slv:
        x0 = _t(s.x).requires_grad_(True)
        q0 = _t(s.quat).requires_grad_(True)
        Ft = _t(F).requires_grad_(True)
        xu, _ = rollout(slv, x0, q0, _glen(s), Ft, checkpoint_every=k, cg_tol=1e-12)
        loss = (xu * xu).sum()
        loss.backward()
        return float(loss), x0.grad.cpu().numpy(), q0.grad.cpu().numpy(), Ft.grad.cpu().numpy()


def test_rollout_matches_oracle(gpu_lib):
    """Three steps of the 20-rod periodic system at volume fraction 0.05,
    checkpoint every 2 steps: gradients of sum |x_unwrapped(T)|^2."""
    s = SYSTEMS["fd20"]()
    rng = np.random.default_rng(11)
    F = np.stack([s.force] + [rng.standard_normal(s.force.shape) for _ in range(2)])
    want = adj.rollout_grad(s.x, s.quat, s.length, F, s.box, s.diam, s.cutoff, s.eta, s.dt)
    loss, gx, gq, gF = _gpu_rollout_grad(gpu_lib, s, F, 2)
    assert loss == pytest.approx(want.loss, rel=1e-9)
    _close("x0_bar", gx, want.x0_bar)
    _close("quat0_bar", gq, want.quat0_bar)
    _close("F_bar", gF, want.F_bar)


def test_checkpointing_is_bitwise(gpu_lib):
    """Recomputed segments reproduce the forward states exactly, so the
    gradient does not depend on the checkpoint interval."""
    s = SYSTEMS["rods200"]()
    rng = np.random.default_rng(12)
    F = np.stack([rng.standard_normal(s.force.shape) for _ in range(5)])
    ref = _gpu_rollout_grad(gpu_lib, s, F, 1)
    for k in (2, 5):
        got = _gpu_rollout_grad(gpu_lib, s, F, k)
        assert got[0] == ref[0]
        for a, b in zip(got[1:], ref[1:]):
            assert np.array_equal(a, b)
