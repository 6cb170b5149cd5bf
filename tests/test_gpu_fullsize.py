"""Parity at the full benchmark size: the 100,000-rod nematic suspension
that bench.py times, through the same entry points and launch shapes.

The expected values were written once by tests/golden/make_rods100k_golden.py
(oracle only): the canonical pair list (as a SHA-256) and U at 500 sampled
rods.  The step's U is also compared over all 6N entries with the oracle's
own solve, run in the test (about 15 s of CPU).  Beside that, the GPU's gamma
is certified with the oracle's own operator: it must satisfy the
complementarity conditions to the tolerance, which pins U (unique for a
convex QP) independently of the stored values."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rods100k_seed0.json")))


@pytest.fixture(scope="module")
def system():
    return rodsynth.cfg_paper_scale(0)


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _solver(rl, s):
    return rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8, max_iter=200_000)


def test_fullsize_pair_list_bit_exact(gpu_lib, system):
    s = system
    d = oracle.directors(s.quat)
    with _solver(gpu_lib, s) as slv:
        pi, pj, img, fl = slv.build_pairs(_t(s.x), _t(d), 1.0)
    assert pi.shape[0] == GOLD["n_pairs"]
    assert GOLD["n_flagged_cutoff"] == 0
    h = hashlib.sha256()
    for a in (pi, pj, img):
        h.update(a.cpu().numpy().astype("<i4").tobytes())
    assert h.hexdigest() == GOLD["pair_sha256"]


@pytest.fixture(scope="module")
def oracle_velocities(system):
    """The oracle's own solve of the whole system (cell-list pairs, BBPGD to
    1e-8; about 15 s of CPU): U over all 6N entries."""
    s = system
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff, method="cells")
    cs = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, s.force)
    r = oracle.bbpgd(d, 1.0, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=200_000)
    assert r.status == oracle.OK
    return oracle.velocity(d, 1.0, s.diam, s.eta, pr, cs, r.gamma, s.force)


def test_fullsize_step_velocities(gpu_lib, system, oracle_velocities):
    s = system
    with _solver(gpu_lib, s) as slv:
        x, q = _t(s.x), _t(s.quat)
        U, info, npairs = slv.step(x, q, 1.0, F=_t(s.force))
    assert npairs == GOLD["n_pairs"]
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    U = U.cpu().numpy()
    # the bar over all 6N entries, against the oracle's solve
    Uo = oracle_velocities
    assert np.linalg.norm(U - Uo) <= 1e-6 * np.linalg.norm(Uo)
    want = np.asarray(GOLD["U_sample"])
    got = U[np.asarray(GOLD["sample_rods"])]
    assert np.linalg.norm(got - want) <= 1e-6 * np.linalg.norm(want)
    assert np.linalg.norm(U) == pytest.approx(GOLD["U_norm"], rel=1e-6)


def test_fullsize_solve_certificate(gpu_lib, system):
    """rl_solve_lcp on the oracle's own constraint geometry; the oracle's
    operator certifies the answer: gamma >= 0, |min(gamma, Mc gamma + q)| <=
    tol, and U = M(D gamma + F) as the oracle computes it from that gamma."""
    s = system
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff, method="cells")
    cs = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, s.force)
    with _solver(gpu_lib, s) as slv:
        g, U, info = slv.solve_lcp(_t(d), 1.0, _t(pr.pi, torch.int32), _t(pr.pj, torch.int32), _t(cs.e),
                                   _t(cs.arm), _t(cs.q), F=_t(s.force))
    g, U = g.cpu().numpy(), U.cpu().numpy()
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    w = oracle.apply_Mc(d, 1.0, s.diam, s.eta, pr, cs, g)
    assert g.min() >= 0.0
    # the two sides round differently: allow 1e-12 relative to |q| on top of tol
    assert np.abs(np.minimum(g, w)).max() <= 1e-8 + 1e-12 * np.abs(cs.q).max()
    Uo = oracle.velocity(d, 1.0, s.diam, s.eta, pr, cs, g, s.force)
    assert np.linalg.norm(U - Uo) <= 1e-12 * np.linalg.norm(Uo)
    want = np.asarray(GOLD["U_sample"])
    assert np.linalg.norm(U[np.asarray(GOLD["sample_rods"])] - want) <= 1e-6 * np.linalg.norm(want)
