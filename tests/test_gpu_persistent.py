"""The persistent schedule of the FP64 loop (rl_set_loop(RL_LOOP_PERSISTENT)):
one cooperative launch per solve, grid barriers between the rod and the
constraint phase.  Its arithmetic per rod and per constraint is that of the
two-launch loop, so it is held to the same bar: the oracle's own operator
certifies the answer (residual <= tol, U = oracle U(gamma)) and U matches the
oracle's solution to 1e-6, at test sizes and at the 100k-rod benchmark size."""
import json
import os

import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rods100k_seed0.json")))


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _length(s):
    return s.uniform_length if s.uniform_length is not None else s.length


def _gpu_length(s):
    return s.uniform_length if s.uniform_length is not None else _t(s.length)


def _setup(s, method="auto"):
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, _length(s), s.box, s.diam, s.cutoff, method=method)
    cs = oracle.assemble(s.x, d, _length(s), s.box, s.diam, s.eta, s.dt, pr, s.force)
    return d, pr, cs


def _solve(rl, s, d, pr, cs, loop):
    with rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8, max_iter=200_000,
                   loop=loop) as slv:
        g, U, info = slv.solve_lcp(_t(d), _gpu_length(s), _t(pr.pi, torch.int32), _t(pr.pj, torch.int32),
                                   _t(cs.e), _t(cs.arm), _t(cs.q), F=_t(s.force))
        prof = slv.profile_read_loop()
    return g.cpu().numpy(), U.cpu().numpy(), info, prof


def _certify(s, d, pr, cs, g, U):
    w = oracle.apply_Mc(d, _length(s), s.diam, s.eta, pr, cs, g)
    assert g.min(initial=0.0) >= 0.0
    assert np.abs(np.minimum(g, w)).max(initial=0.0) <= 1e-8 + 1e-12 * np.abs(cs.q).max(initial=1.0)
    Uo = oracle.velocity(d, _length(s), s.diam, s.eta, pr, cs, g, s.force)
    assert np.linalg.norm(U - Uo) <= 1e-12 * np.linalg.norm(Uo)


@pytest.mark.parametrize("which", ["small", "lengths", "dense10k", "hub"])
def test_persistent_matches_oracle(gpu_lib, which):
    s = {"small": lambda: rodsynth.cfg_small(0), "hub": lambda: rodsynth.cfg_hub(1),
         "lengths": lambda: rodsynth.make_system(1000, seed=1, phi=0.04, length=(0.5, 1.5)),
         "dense10k": lambda: rodsynth.cfg_paper_scale(0, n=10_000)}[which]()
    d, pr, cs = _setup(s)
    g, U, info, prof = _solve(gpu_lib, s, d, pr, cs, gpu_lib.LOOP_PERSISTENT)
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    assert prof["launches"] == 1 and prof["iterations"] == info.iterations
    _certify(s, d, pr, cs, g, U)
    ref = oracle.bbpgd(d, _length(s), s.diam, s.eta, pr, cs, tol=1e-8)
    Uref = oracle.velocity(d, _length(s), s.diam, s.eta, pr, cs, ref.gamma, s.force)
    assert np.linalg.norm(U - Uref) <= 1e-6 * np.linalg.norm(Uref)
    # the two schedules solve the same problem
    g2, U2, info2, prof2 = _solve(gpu_lib, s, d, pr, cs, gpu_lib.LOOP_LAUNCH)
    assert prof2["launches"] == 0
    assert np.linalg.norm(U - U2) <= 1e-6 * np.linalg.norm(U2)


def test_persistent_bitwise_repeatable(gpu_lib):
    s = rodsynth.cfg_paper_scale(0, n=10_000)
    d, pr, cs = _setup(s)
    a = _solve(gpu_lib, s, d, pr, cs, gpu_lib.LOOP_PERSISTENT)
    b = _solve(gpu_lib, s, d, pr, cs, gpu_lib.LOOP_PERSISTENT)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2].iterations == b[2].iterations


def test_persistent_fullsize(gpu_lib):
    """The 100k-rod benchmark step (rl_step renumbers the rods in cell order,
    so every block of rods has both P- and Q-side records to spare): U at the
    sampled rods against the oracle's stored values."""
    s = rodsynth.cfg_paper_scale(0)
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8, max_iter=200_000,
                        loop=gpu_lib.LOOP_PERSISTENT) as slv:
        U, info, npairs = slv.step(_t(s.x), _t(s.quat), 1.0, F=_t(s.force))
        prof = slv.profile_read_loop()
    assert npairs == GOLD["n_pairs"] and prof["launches"] == 1
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    U = U.cpu().numpy()
    want = np.asarray(GOLD["U_sample"])
    assert np.linalg.norm(U[np.asarray(GOLD["sample_rods"])] - want) <= 1e-6 * np.linalg.norm(want)
    assert np.linalg.norm(U) == pytest.approx(GOLD["U_norm"], rel=1e-6)


def test_persistent_reports_what_does_not_fit(gpu_lib):
    """Rods in a random order: with pi <= pj the low-numbered rods hold almost
    only P-side records and the high-numbered ones Q-side records, so no split
    into one block per compute unit fits the LDS; the solve says so."""
    s = rodsynth.cfg_paper_scale(0)
    d, pr, cs = _setup(s, method="cells")
    with pytest.raises(gpu_lib.RodLCPError, match="does not fit"):
        _solve(gpu_lib, s, d, pr, cs, gpu_lib.LOOP_PERSISTENT)


def test_persistent_step_and_empty(gpu_lib):
    s = rodsynth.cfg_small(0)
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8,
                        loop=gpu_lib.LOOP_PERSISTENT) as slv:
        U, info, npairs = slv.step(_t(s.x), _t(s.quat), 1.0, F=_t(s.force))
        assert info.status == gpu_lib.OK and npairs > 0
    # no constraints: U = M F, no launch of the loop
    far = rodsynth.make_system(50, seed=3, box=60.0)
    with gpu_lib.Solver(box=far.box, diam=far.diam, cutoff=far.cutoff, eta=far.eta, dt=far.dt, tol=1e-8,
                        loop=gpu_lib.LOOP_PERSISTENT) as slv:
        U0, info0, n0 = slv.step(_t(far.x), _t(far.quat), 1.0, F=_t(far.force))
        assert n0 == 0 and info0.iterations == 0 and slv.profile_read_loop()["launches"] == 0
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8) as slv:
        U2, info2, _ = slv.step(_t(s.x), _t(s.quat), 1.0, F=_t(s.force))
    U, U2 = U.cpu().numpy(), U2.cpu().numpy()
    assert np.linalg.norm(U - U2) <= 1e-6 * np.linalg.norm(U2)


def test_loop_mode_is_checked(gpu_lib):
    with gpu_lib.Solver(box=4.0) as slv:
        with pytest.raises(gpu_lib.RodLCPError):
            slv.set_loop(7)
