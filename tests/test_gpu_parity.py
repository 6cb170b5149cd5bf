"""Parity of the HIP library (through its C-ABI) with the CPU FP64 oracle.

Bars: the pair list is bit-exact after the canonical order, except pairs
flagged within 1e-9 of the threshold; phi, e, arm and q agree to 1e-12
(relative to the magnitude of q for q); Mc gamma + q to 1e-12 relative;
velocities U = M(D gamma + F) to 1e-6 relative (2-norm over all rods) with
both residuals <= 1e-8, because gamma need not be unique while U is."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _solver(rl, s, **kw):
    kw.setdefault("tol", 1e-8)
    return rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, **kw)


def _length(s):
    return s.uniform_length if s.uniform_length is not None else s.length


def _gpu_length(s):
    return s.uniform_length if s.uniform_length is not None else _t(s.length)


def _gpu_pairs(rl, slv, s, d_gpu):
    pi, pj, img, fl = slv.build_pairs(_t(s.x), d_gpu, _gpu_length(s))
    return (pi.cpu().numpy(), pj.cpu().numpy(), img.cpu().numpy(), fl.cpu().numpy())


def _assert_pairs_match(got, want: oracle.Pairs):
    gkey = set(zip(got[0].tolist(), got[1].tolist(), got[2].tolist()))
    wkey = set(zip(want.pi.tolist(), want.pj.tolist(), want.img.tolist()))
    flagged = {k for k, f in zip(zip(want.pi.tolist(), want.pj.tolist(), want.img.tolist()), want.flags.tolist())
               if f & oracle.FLAG_CUTOFF}
    flagged |= {k for k, f in zip(zip(*[g.tolist() for g in got[:3]]), got[3].tolist()) if f & oracle.FLAG_CUTOFF}
    assert (gkey ^ wkey) <= flagged
    if not flagged:
        assert np.array_equal(got[0], want.pi) and np.array_equal(got[1], want.pj)
        assert np.array_equal(got[2], want.img)
        assert np.array_equal(got[3] & ~np.uint8(oracle.FLAG_PARALLEL), want.flags & ~np.uint8(oracle.FLAG_PARALLEL))
    # canonical order
    key = got[0].astype(np.int64) * (1 << 40) + got[1].astype(np.int64) * (1 << 12) + got[2]
    assert np.all(np.diff(key) > 0)


def test_directors(gpu_lib):
    rng = np.random.default_rng(0)
    q = rng.standard_normal((1000, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    with _solver(gpu_lib, rodsynth.cfg_small(0)) as slv:
        d = slv.directors(_t(q)).cpu().numpy()
    assert np.allclose(d, oracle.directors(q), rtol=0, atol=2e-16 * 4)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pairs_small_config(gpu_lib, seed):
    s = rodsynth.cfg_small(seed)
    d = oracle.directors(s.quat)
    want = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff, method="brute")
    with _solver(gpu_lib, s) as slv:
        got = _gpu_pairs(gpu_lib, slv, s, _t(d))
    _assert_pairs_match(got, want)


@pytest.mark.parametrize("n,phi,length", [(200, 0.1, 1.0), (60, 0.1, 1.0), (120, 0.02, 1.0),
                                          (700, 0.08, (0.5, 1.5)), (333, 0.05, 1.0)])
def test_pairs_small_boxes_and_lengths(gpu_lib, n, phi, length):
    s = rodsynth.make_system(n, seed=n, phi=phi, length=length)
    d = oracle.directors(s.quat)
    want = oracle.pairs(s.x, d, _length(s), s.box, s.diam, s.cutoff, method="brute")
    with _solver(gpu_lib, s) as slv:
        got = _gpu_pairs(gpu_lib, slv, s, _t(d))
    _assert_pairs_match(got, want)


@pytest.mark.parametrize("seed", [0, 1])
def test_pairs_hub(gpu_lib, seed):
    """One rod of length 4 among 36 crossing rods in a box of 10 (two cells
    per side, so the stencil wraps onto the same cells): the pair list is the
    brute force's, bit for bit."""
    s = rodsynth.cfg_hub(seed)
    d = oracle.directors(s.quat)
    want = oracle.pairs(s.x, d, s.length, s.box, s.diam, s.cutoff, method="brute")
    assert np.sum(want.pi == 18) == 18 and np.sum(want.pj == 18) == 18
    with _solver(gpu_lib, s) as slv:
        got = _gpu_pairs(gpu_lib, slv, s, _t(d))
    _assert_pairs_match(got, want)


def test_pairs_hand_cases(gpu_lib):
    def q_for(v):
        v = np.asarray(v, float) / np.linalg.norm(v)
        q = np.r_[1.0 + v[2], np.cross([0, 0, 1.0], v)]
        return q / np.linalg.norm(q)
    # across the periodic boundary
    x = np.array([[0.02, 2.0, 2.0], [3.99, 2.0, 2.03]])
    d = oracle.directors(np.stack([q_for([0, 1, 0]), q_for([0, 0, 1])]))
    s = rodsynth.make_system(2, seed=0, box=4.0)
    with _solver(gpu_lib, s) as slv:
        got = _gpu_pairs(gpu_lib, slv, rodsynth.RodSystem(x, s.quat, s.length, s.force, 4.0), _t(d))
    assert got[0].tolist() == [0] and got[1].tolist() == [1] and got[2].tolist() == [oracle.img_pack(-1, 0, 0)]
    # a rod touching its own image (parallel axes: midpoint rule)
    x = np.array([[0.5, 0.5, 0.5]])
    d = oracle.directors(q_for([1, 0, 0])[None])
    s = rodsynth.make_system(1, seed=0, box=1.04)
    with _solver(gpu_lib, s) as slv:
        got = _gpu_pairs(gpu_lib, slv, rodsynth.RodSystem(x, s.quat, s.length, s.force, 1.04), _t(d))
        phi, e, arm, q = slv.assemble_D(_t(x), _t(d), 1.0, *[_t(v, torch.int32) for v in got[:3]],
                                        _t(np.zeros((1, 6))))
    assert got[0].tolist() == [0] and got[1].tolist() == [0] and got[2].tolist() == [oracle.img_pack(1, 0, 0)]
    pr = oracle.Pairs(*[np.asarray(v) for v in got])
    cs = oracle.assemble(x, d, 1.0, 1.04, 0.025, 0.01, 1e-4, pr, np.zeros((1, 6)))
    assert np.allclose(phi.cpu().numpy(), cs.phi, atol=1e-15)
    assert np.allclose(arm.cpu().numpy(), cs.arm, atol=1e-15)


def _c6_cases():
    """Pairs that take the closest-point fallbacks, one pair per case, each
    case far from the others (box 24, cases 4 apart).  Directors are given
    exactly (axis-aligned or simple), so both sides see the same inputs.
      0 axes crossing at both centres (dist 0: e = +d_i x d_j)
      1 axes crossing off-centre (s = 0.25 on rod 0)
      2 axes 5e-13 apart (below the degenerate distance): e = -z, the sign
        of r0 along d_i x d_j
      3 collinear, overlapping end to end (e from the least-aligned axis)
      4 collinear, antiparallel
      5 parallel side by side, interior overlap (midpoint rule)
      6 parallel, not overlapping along the axis (end points)
      7 near-parallel (tilt 1e-9 rad: 1 - b^2 below the parallel band)
    """
    X, D = [], []
    ex, ey, ez = np.eye(3)
    c = lambda k: np.array([2.0 + 4.0 * (k % 5), 2.0 + 4.0 * (k // 5), 12.0])  # noqa: E731
    cases = [
        ((0, 0, 0), ex, (0, 0, 0), ey),
        ((0, 0, 0), ex, (0.25, 0, 0), ey),
        ((0, 0, 0), ex, (0.25, 0, 5e-13), ey),
        ((0, 0, 0), ex, (0.5, 0, 0), ex),
        ((0, 0, 0), ex, (0.75, 0, 0), -ex),
        ((0, 0, 0), ex, (0.3, 0.02, 0), ex),
        ((0, 0, 0), ex, (1.01, 0.01, 0), ex),
        ((0, 0, 0), ex, (0.3, 0.02, 0), np.array([1.0, 1e-9, 0.0]) / math.hypot(1.0, 1e-9)),
    ]
    for k, (x0, d0, x1, d1) in enumerate(cases):
        X += [c(k) + np.asarray(x0, float), c(k) + np.asarray(x1, float)]
        D += [np.asarray(d0, float), np.asarray(d1, float)]
    return np.array(X), np.array(D)


def test_closest_point_fallbacks_match_the_oracle(gpu_lib):
    """The parallel, intersecting and collinear fallbacks change D and U, so
    the GPU must take the same choices as the oracle: pairs, flags, gaps,
    normals, lever arms and q compared element by element with no mask, then
    the solve's velocities."""
    x, d = _c6_cases()
    n = x.shape[0]
    rng = np.random.default_rng(8)
    F = rng.standard_normal((n, 6))
    box = 24.0
    s = rodsynth.make_system(n, seed=0, box=box)
    s = rodsynth.RodSystem(x=x, quat=s.quat, length=np.ones(n), force=F, box=box)
    pr = oracle.pairs(x, d, 1.0, box, s.diam, s.cutoff)
    cs = oracle.assemble(x, d, 1.0, box, s.diam, s.eta, s.dt, pr, F)
    assert pr.n == 8 and np.array_equal(pr.pi, np.arange(0, n, 2)) and np.array_equal(pr.pj, pr.pi + 1)
    assert np.all(pr.flags[[0, 1, 2, 3, 4]] & oracle.FLAG_DEGENERATE)
    assert np.all(pr.flags[[3, 4, 5, 6, 7]] & oracle.FLAG_PARALLEL)
    assert np.array_equal(cs.e[0], [0.0, 0.0, 1.0]) and np.array_equal(cs.e[2], [0.0, 0.0, -1.0])
    assert np.array_equal(cs.arm[1], [0.25, 0.0]) and np.allclose(cs.arm[5], [0.15, -0.15], atol=1e-15)
    with _solver(gpu_lib, s) as slv:
        got = _gpu_pairs(gpu_lib, slv, s, _t(d))
        assert np.array_equal(got[0], pr.pi) and np.array_equal(got[1], pr.pj)
        assert np.array_equal(got[2], pr.img) and np.array_equal(got[3], pr.flags)
        phi, e, arm, q = slv.assemble_D(_t(x), _t(d), 1.0, *[_t(v, torch.int32) for v in got[:3]], _t(F))
        phi, e, arm, q = (v.cpu().numpy() for v in (phi, e, arm, q))
        assert np.abs(phi - cs.phi).max() <= 1e-15
        assert np.abs(e - cs.e).max() <= 1e-15
        assert np.abs(arm - cs.arm).max() <= 1e-15
        assert np.abs(q - cs.q).max() <= 1e-12 * np.abs(cs.q).max()
        g, U, info = slv.solve_lcp(_t(d), 1.0, _t(pr.pi, torch.int32), _t(pr.pj, torch.int32), _t(cs.e),
                                   _t(cs.arm), _t(cs.q), F=_t(F))
    assert info.status == gpu_lib.OK
    ref = oracle.bbpgd(d, 1.0, s.diam, s.eta, pr, cs, tol=1e-8)
    Uo = oracle.velocity(d, 1.0, s.diam, s.eta, pr, cs, ref.gamma, F)
    assert np.linalg.norm(U.cpu().numpy() - Uo) <= 1e-6 * np.linalg.norm(Uo)


def test_pairs_capacity_and_errors(gpu_lib):
    s = rodsynth.cfg_small(0)
    d = _t(oracle.directors(s.quat))
    with _solver(gpu_lib, s) as slv:
        with pytest.raises(gpu_lib.RodLCPError) as ei:
            slv.build_pairs(_t(s.x), d, 1.0, capacity=10)
        assert ei.value.status == gpu_lib.ERR_CAPACITY
        xbad = s.x.copy()
        xbad[3, 1] = s.box + 0.1
        with pytest.raises(gpu_lib.RodLCPError) as ei:
            slv.build_pairs(_t(xbad), d, 1.0)
        assert ei.value.status == gpu_lib.ERR_ARG
        xbad[3, 1] = float("nan")
        with pytest.raises(gpu_lib.RodLCPError) as ei:
            slv.build_pairs(_t(xbad), d, 1.0)
        assert ei.value.status == gpu_lib.ERR_NONFINITE


def _geometry_tolerance(s, d, pr, cs):
    """Per-pair bars for the normal and the lever arms.  The closest-point
    problem amplifies rounding: the arms move by ~u L / (1 - b^2) and the
    normal by ~u L / ((1 - b^2) dist) for a relative input change u (measured
    on the oracle itself: <= 1.3e-15 L/((1-b^2) dist) under 1-ulp input
    changes).  Bars: 1e-12 plus 1e-14 times those factors."""
    L = np.maximum(s.length[pr.pi], s.length[pr.pj])
    b = np.einsum("ij,ij->i", d[pr.pi], d[pr.pj])
    den = np.maximum(1.0 - b * b, 1e-10)
    dist = np.maximum(cs.phi + s.diam, 1e-12)
    return 1e-12 + 1e-14 * L / (den * dist), 1e-12 + 1e-14 * L / den


def _oracle_setup(s):
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, _length(s), s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, _length(s), s.box, s.diam, s.eta, s.dt, pr, s.force)
    return d, pr, cs


@pytest.mark.parametrize("which", ["small", "lengths"])
def test_assemble(gpu_lib, which):
    s = rodsynth.cfg_small(3) if which == "small" else rodsynth.make_system(900, seed=4, phi=0.08, length=(0.5, 1.5))
    d, pr, cs = _oracle_setup(s)
    with _solver(gpu_lib, s) as slv:
        phi, e, arm, q = slv.assemble_D(_t(s.x), _t(d), _gpu_length(s), _t(pr.pi, torch.int32),
                                        _t(pr.pj, torch.int32), _t(pr.img, torch.int32), _t(s.force))
    ok = (pr.flags & (oracle.FLAG_PARALLEL | oracle.FLAG_DEGENERATE)) == 0
    tol_e, tol_arm = _geometry_tolerance(s, d, pr, cs)
    assert np.allclose(phi.cpu().numpy(), cs.phi, rtol=0, atol=1e-12)
    assert np.all(np.abs(e.cpu().numpy() - cs.e).max(axis=1)[ok] <= tol_e[ok])
    assert np.all(np.abs(arm.cpu().numpy() - cs.arm).max(axis=1)[ok] <= tol_arm[ok])
    # q = phi/h + D^T M F inherits the geometry tolerance through the free velocities
    Unc = oracle.apply_mobility(d, _length(s), s.diam, s.eta, s.force)
    ut, wr = np.abs(Unc[:, :3]).max(), np.abs(Unc[:, 3:]).max()
    Lmax = np.max(s.length)
    tol_q = 1e-12 * np.abs(cs.q).max() + 4 * (ut + wr * Lmax) * tol_e + 4 * wr * tol_arm
    assert np.all(np.abs(q.cpu().numpy() - cs.q)[ok] <= tol_q[ok])
    assert np.abs(q.cpu().numpy() - cs.q).max() <= 1e-9 * np.abs(cs.q).max()


@pytest.mark.parametrize("which", ["small", "lengths"])
def test_apply_M(gpu_lib, which):
    s = rodsynth.cfg_small(1) if which == "small" else rodsynth.make_system(900, seed=4, phi=0.08, length=(0.5, 1.5))
    d, pr, cs = _oracle_setup(s)
    gamma = np.abs(np.random.default_rng(0).standard_normal(pr.n))
    want = oracle.apply_Mc(d, _length(s), s.diam, s.eta, pr, cs, gamma)
    with _solver(gpu_lib, s) as slv:
        w = slv.apply_M(_t(d), _gpu_length(s), _t(pr.pi, torch.int32), _t(pr.pj, torch.int32), _t(cs.e),
                        _t(cs.arm), _t(cs.q), _t(gamma)).cpu().numpy()
    assert np.abs(w - want).max() <= 1e-12 * np.abs(want).max()


def _gpu_solve(gpu_lib, s, d, pr, cs, **kw):
    with _solver(gpu_lib, s, **kw) as slv:
        g, U, info = slv.solve_lcp(_t(d), _gpu_length(s), _t(pr.pi, torch.int32), _t(pr.pj, torch.int32),
                                   _t(cs.e), _t(cs.arm), _t(cs.q), F=_t(s.force))
    return g.cpu().numpy(), U.cpu().numpy(), info


def _assert_dense(s, pr):
    """The system takes the rod kernels' dense form (above 8 constraints per
    rod: eight lanes per rod, three rounds of records each), and some rods
    have more than the 24 records a side that the rounds hold, so the loop
    past them runs too."""
    assert pr.n > 8 * s.n
    assert np.bincount(pr.pi, minlength=s.n).max() > 24 and np.bincount(pr.pj, minlength=s.n).max() > 24


def _phi08():
    # relaxed isotropic suspension at the precision workload's density
    return rodsynth.relaxed_system(1500, seed=3, phi=0.08, length=(0.5, 1.5))


@pytest.mark.parametrize("which", ["small0", "small1", "lengths", "dense10k", "hub", "phi08"])
def test_solve_matches_oracle(gpu_lib, which):
    s = {"small0": lambda: rodsynth.cfg_small(0), "small1": lambda: rodsynth.cfg_small(1),
         "hub": lambda: rodsynth.cfg_hub(1),
         "lengths": lambda: rodsynth.make_system(1000, seed=1, phi=0.04, length=(0.5, 1.5)),
         "dense10k": lambda: rodsynth.cfg_paper_scale(0, n=10_000), "phi08": _phi08}[which]()
    d, pr, cs = _oracle_setup(s)
    if which == "phi08":
        _assert_dense(s, pr)
    ref = oracle.bbpgd(d, _length(s), s.diam, s.eta, pr, cs, tol=1e-8)
    Uref = oracle.velocity(d, _length(s), s.diam, s.eta, pr, cs, ref.gamma, s.force)
    g, U, info = _gpu_solve(gpu_lib, s, d, pr, cs)
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    # certificate of the GPU answer with the oracle's own operator
    w = oracle.apply_Mc(d, _length(s), s.diam, s.eta, pr, cs, g)
    assert g.min() >= 0 and np.abs(np.minimum(g, w)).max() <= 1e-8 * 1.01
    assert np.linalg.norm(U - Uref) <= 1e-6 * np.linalg.norm(Uref)
    # BB is non-monotone, so rounding differences change the path after a
    # while; the counts stay of the same size (early iterates are compared
    # exactly in test_early_iterates_match)
    assert 0.5 * ref.iterations <= info.iterations <= 2.0 * ref.iterations


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_early_iterates_match(gpu_lib, k):
    """The first BBPGD iterates (same start, same Cauchy step, same BB rule)
    agree before rounding differences are amplified."""
    s = rodsynth.cfg_paper_scale(0, n=10_000)
    d, pr, cs = _oracle_setup(s)
    ref = oracle.bbpgd(d, 1.0, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=k)
    g, U, info = _gpu_solve(gpu_lib, s, d, pr, cs, max_iter=k)
    assert info.iterations == ref.iterations == k
    assert info.alpha0 == pytest.approx(ref.alpha0, rel=1e-12)
    assert np.abs(g - ref.gamma).max() <= 1e-9 * np.abs(ref.gamma).max()
    assert info.residual == pytest.approx(ref.residual, rel=1e-8)


def test_infeasible_system_is_reported(gpu_lib):
    """900 rods up to 1.5 long at volume fraction 0.08 in a periodic box of
    1.78: the linearised problem has no solution (the oracle's objective
    falls without bound).  Both sides must say so instead of returning a
    'solution'."""
    s = rodsynth.make_system(900, seed=4, phi=0.08, length=(0.5, 1.5))
    d, pr, cs = _oracle_setup(s)
    ref = oracle.bbpgd(d, s.length, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=3000)
    g, U, info = _gpu_solve(gpu_lib, s, d, pr, cs, max_iter=3000)
    assert ref.status == oracle.NOT_CONVERGED and info.status == gpu_lib.NOT_CONVERGED
    assert info.iterations == 3000 and ref.residual > 1.0 and info.residual > 1.0


def test_solve_two_rod_closed_form(gpu_lib):
    diam, eta, dt = 0.025, 0.01, 1e-4
    gap = -0.005
    s = rodsynth.make_system(2, seed=0, box=50.0)
    s.x[:] = [[5, 5, 5 + diam + gap], [5, 5, 5]]
    s.quat[0] = np.array([1, 0, 1, 0]) / math.sqrt(2)     # along x
    s.quat[1] = np.array([1, -1, 0, 0]) / math.sqrt(2)    # along y
    s.force[:] = 0.0
    s.force[0, 2], s.force[1, 2] = -2.0, 3.0
    d, pr, cs = _oracle_setup(s)
    assert pr.n == 1
    g, U, info = _gpu_solve(gpu_lib, s, d, pr, cs)
    a = oracle.mobility_coeffs(1.0, diam, eta)
    q = gap / dt + a[1] * (-2.0 - 3.0)
    assert g[0] == pytest.approx(max(0.0, -q / (2 * a[1])), rel=1e-12)
    assert U[0, 2] - U[1, 2] == pytest.approx(-gap / dt, rel=1e-12)
    assert info.iterations == 1


def test_solve_edge_cases(gpu_lib):
    s = rodsynth.make_system(300, seed=2, box=30.0)   # dilute: few or no contacts
    d, pr, cs = _oracle_setup(s)
    g, U, info = _gpu_solve(gpu_lib, s, d, pr, cs)
    Uref = oracle.velocity(d, 1.0, s.diam, s.eta, pr, cs, oracle.bbpgd(d, 1.0, s.diam, s.eta, pr, cs).gamma, s.force)
    assert np.allclose(U, Uref, rtol=1e-12, atol=1e-10)
    # no constraints at all: U = M F
    empty = oracle.Pairs(*(np.zeros(0, np.int32),) * 3, np.zeros(0, np.uint8))
    ce = oracle.Constraints(np.zeros(0), np.zeros((0, 3)), np.zeros((0, 2)), np.zeros(0))
    g, U, info = _gpu_solve(gpu_lib, s, d, empty, ce)
    assert info.iterations == 0 and info.status == gpu_lib.OK
    assert np.allclose(U, oracle.apply_mobility(d, 1.0, s.diam, s.eta, s.force), rtol=1e-14, atol=1e-12)


def test_solve_status_codes(gpu_lib):
    s = rodsynth.cfg_small(0)
    d, pr, cs = _oracle_setup(s)
    g, U, info = _gpu_solve(gpu_lib, s, d, pr, cs, max_iter=1)
    assert info.status == gpu_lib.NOT_CONVERGED and info.iterations == 1
    ref = oracle.bbpgd(d, 1.0, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=1)
    assert info.residual == pytest.approx(ref.residual, rel=1e-9)
    bad = oracle.Constraints(cs.phi, cs.e, cs.arm, cs.q.copy())
    bad.q[5] = float("nan")
    with pytest.raises(gpu_lib.RodLCPError) as ei:
        _gpu_solve(gpu_lib, s, d, pr, bad)
    assert ei.value.status == gpu_lib.ERR_NONFINITE
    unsorted = oracle.Pairs(pr.pi[::-1].copy(), pr.pj[::-1].copy(), pr.img, pr.flags)
    with pytest.raises(gpu_lib.RodLCPError) as ei:
        _gpu_solve(gpu_lib, s, d, unsorted, cs)
    assert ei.value.status == gpu_lib.ERR_ARG
    oob = oracle.Pairs(pr.pi, pr.pj.copy(), pr.img, pr.flags)
    oob.pj[-1] = s.n
    with pytest.raises(gpu_lib.RodLCPError) as ei:
        _gpu_solve(gpu_lib, s, d, oob, cs)
    assert ei.value.status == gpu_lib.ERR_ARG


def test_solve_bitwise_repeatable(gpu_lib):
    s = rodsynth.cfg_paper_scale(1, n=5000)
    d, pr, cs = _oracle_setup(s)
    g1, U1, i1 = _gpu_solve(gpu_lib, s, d, pr, cs)
    g2, U2, i2 = _gpu_solve(gpu_lib, s, d, pr, cs)
    assert i1.iterations == i2.iterations
    assert np.array_equal(g1, g2) and np.array_equal(U1, U2)


@pytest.mark.parametrize("which", ["small", "lengths", "hub", "phi08"])
def test_step_matches_oracle(gpu_lib, which):
    """"hub": one rod 4 long in a box of 10 (two cells per side) with 18
    contacts on each side of its incidence lists; "phi08": 12 constraints
    per rod."""
    s = {"small": lambda: rodsynth.cfg_small(5),
         "lengths": lambda: rodsynth.make_system(800, seed=6, phi=0.06, length=(0.5, 1.5)),
         "hub": lambda: rodsynth.cfg_hub(1), "phi08": _phi08}[which]()
    r = oracle.step_solve(s)
    if which == "phi08":
        _assert_dense(s, r.pairs)
    xo, qo = s.x.copy(), s.quat.copy()
    oracle.integrate(s.box, s.dt, r.U, xo, qo)
    x, quat = _t(s.x), _t(s.quat)
    with _solver(gpu_lib, s) as slv:
        U, info, npairs = slv.step(x, quat, _gpu_length(s), F=_t(s.force))
    assert npairs == r.pairs.n
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    U = U.cpu().numpy()
    assert np.linalg.norm(U - r.U) <= 1e-6 * np.linalg.norm(r.U)
    # the state moves by h U, so it inherits the velocity tolerance
    bound = 1e-6 * s.dt * np.linalg.norm(r.U) + 1e-14
    dx = (x.cpu().numpy() - xo + 0.5 * s.box) % s.box - 0.5 * s.box
    assert np.abs(dx).max() <= bound
    assert np.abs(quat.cpu().numpy() - qo).max() <= bound


def test_step_empty(gpu_lib):
    s = rodsynth.cfg_small(0)
    with _solver(gpu_lib, s) as slv:
        x = torch.zeros((0, 3), dtype=torch.float64, device=DEV)
        q = torch.zeros((0, 4), dtype=torch.float64, device=DEV)
        U, info, npairs = slv.step(x, q, 1.0, F=torch.zeros((0, 6), dtype=torch.float64, device=DEV))
    assert npairs == 0 and info.status == gpu_lib.OK


def test_reserve_and_params(gpu_lib):
    """rl_reserve pre-sizes the workspace without changing any result, and
    rl_set_params / rl_get_params round-trip (a changed tolerance is used)."""
    s = rodsynth.cfg_small(2)
    outs = []
    for reserve in (False, True):
        with _solver(gpu_lib, s) as slv:
            if reserve:
                slv.reserve(20_000, 200_000)
            U, info, npairs = slv.step(_t(s.x), _t(s.quat), 1.0, F=_t(s.force))
            outs.append((U.cpu().numpy(), info.iterations, npairs))
    assert outs[0][2] == outs[1][2] and outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])
    with _solver(gpu_lib, s) as slv:
        slv.set_params(tol=1e-4)
        got = type(slv.params)()
        assert gpu_lib.load().rl_get_params(slv._h, ctypes.byref(got)) == 0
        assert got.tol == 1e-4 and got.diam == s.diam
        _, info, _ = slv.step(_t(s.x), _t(s.quat), 1.0, F=_t(s.force))
    # the same iterates as with 1e-8, stopped at the first one within 1e-4
    assert info.status == gpu_lib.OK and info.residual <= 1e-4 and info.iterations <= outs[0][1]
